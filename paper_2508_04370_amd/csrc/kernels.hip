// Device kernels of the multifrontal LDL^T (gfx950, wave64).
//
// Front storage: each supernode s owns a dense f x f column-major block (ld = f) in one
// arena.  After factorisation its first p columns hold L (rows in pivoted order) and the
// lower part of F[p:, p:] holds the contribution block (Schur complement) that the
// parent pulls through the child->parent row map (Section 4.1).
//
// Pivoting (Section 4.5) runs in one wavefront on an LDS copy of the window's diagonal
// block B_D: presort swap, Bunch-Kaufman variant with lift, static regularisation added
// after the decision, Proposition 3 and the sign rule (Section 4.6), 1x1 or 2x2 pivots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "device.hpp"

namespace qdmf {

namespace {


typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d16 __attribute__((ext_vector_type(16)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Wave64 reductions with DPP: row_shr 1/2/4/8 leave each row's total in its lane 15,
// row_bcast15 / row_bcast31 combine the four rows into lane 63, which is read back as a
// wave-uniform value.  No LDS round trips.  All 64 lanes must be active.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_shift(double v, double old) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(old), __double2loint(v), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(old), __double2hiint(v), CTRL, ROWMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double lane63(double v) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

__device__ inline double wave_max(double v) {
    v = fmax(v, dpp_shift<0x111, 0xf>(v, v));
    v = fmax(v, dpp_shift<0x112, 0xf>(v, v));
    v = fmax(v, dpp_shift<0x114, 0xf>(v, v));
    v = fmax(v, dpp_shift<0x118, 0xf>(v, v));
    v = fmax(v, dpp_shift<0x142, 0xa>(v, v));
    v = fmax(v, dpp_shift<0x143, 0xc>(v, v));
    return lane63(v);
}

__device__ inline double wave_sum_d(double v) {
    v += dpp_shift<0x111, 0xf>(v, 0.0);
    v += dpp_shift<0x112, 0xf>(v, 0.0);
    v += dpp_shift<0x114, 0xf>(v, 0.0);
    v += dpp_shift<0x118, 0xf>(v, 0.0);
    v += dpp_shift<0x142, 0xa>(v, 0.0);
    v += dpp_shift<0x143, 0xc>(v, 0.0);
    return lane63(v);
}

__device__ inline int wave_sum(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return __builtin_amdgcn_readlane(v, 63);
}

// Maximum value and the lowest lane holding it (lane = position).
__device__ inline void wave_argmax(double v, int /*lane*/, double& bv, int& bi) {
    bv = wave_max(v);
    const unsigned long long m = __ballot(v == bv);
    bi = __ffsll((long long)m) - 1;
}

// LDS state of the one-wave pivot kernel of small fronts: T holds the whole symmetric front
// (f <= FM <= 64), T[i][j] at j*LDW + i.  Sized per launch (FM = 16, 32 or 64) so that the
// many tiny fronts of the lowest levels leave room for many workgroups per CU.
template <int FM>
struct PivShared {
    static constexpr int LDW = FM + 1;
    double T[FM * LDW];
    double sh[FM];  // static shift of the row (-rho primal, +delta dual)
    double w0[FM], w1[FM];
    double d[FM], doff[FM], ed[FM];
    int sg[FM];     // expected pivot sign
    int pm[FM];     // original position now at this position
    int pt[FM], fl[FM], zs[FM];
};

// Symmetric interchange of positions a and b: rows and columns of the symmetric block.
template <int FM>
__device__ void sym_swap(PivShared<FM>& S, int nsym, int a, int b, int lane) {
    constexpr int LDW = PivShared<FM>::LDW;
    if (a == b) return;
    if (lane < nsym) {  // rows a and b of the symmetric block (lane = column)
        double t = S.T[lane * LDW + a];
        S.T[lane * LDW + a] = S.T[lane * LDW + b];
        S.T[lane * LDW + b] = t;
    }
    __syncthreads();
    if (lane < nsym) {  // columns a and b (lane = row)
        double t = S.T[a * LDW + lane];
        S.T[a * LDW + lane] = S.T[b * LDW + lane];
        S.T[b * LDW + lane] = t;
    }
    if (lane == 0) {
        int ts = S.sg[a]; S.sg[a] = S.sg[b]; S.sg[b] = ts;
        double tz = S.sh[a]; S.sh[a] = S.sh[b]; S.sh[b] = tz;
        int tp = S.pm[a]; S.pm[a] = S.pm[b]; S.pm[b] = tp;
    }
    __syncthreads();
}

// T[row][j] -= m * S.w0[j] for j in [j0, ncols): 8 columns per trip so the LDS loads of a
// trip are independent of its stores and can be issued together.
template <int FM>
__device__ inline void rank1_rows(PivShared<FM>& S, int j0, int ncols, double m0, int lane) {
    constexpr int LDW = PivShared<FM>::LDW;
    if (lane >= FM) return;
    for (int jb = j0 & ~7; jb < ncols; jb += 8) {
        double t0[8], w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = jb + q;
            const bool on = j >= j0 && j < ncols;
            w[q] = on ? S.w0[j] : 0.0;
            t0[q] = S.T[j * LDW + lane];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            S.T[(jb + q) * LDW + lane] = t0[q] - m0 * w[q];
        }
    }
}

// Partial LDL^T over the window [0, nbw) of the nsym x nsym symmetric block in S.T, with
// the updates applied to the columns [0, ncols) of the symmetric rows (nsym = ncols).  Pivot
// tests read only the window (Section 4.5).  One wavefront (blockDim.x == 64); every
// decision is wave-uniform.
template <int FM>
__device__ void factor_window(PivShared<FM>& S, int nsym, int nbw, double knorm, const PivotParams& pp,
                              int lane) {
    constexpr int LDW = PivShared<FM>::LDW;
    const int ncols = nsym;
    const double tiny = pp.eps_lift * knorm;  // delta * ||M||_1 of the lift test
    const double alpha = pp.alpha;
    int k = 0;
    while (k < nbw) {
        if (pp.presort) {  // largest |diagonal| of the window to position k
            double v = (lane >= k && lane < nbw) ? fabs(S.T[lane * LDW + lane]) : -1.0;
            double bv;
            int q;
            wave_argmax(v, lane, bv, q);
            if (q < k || q >= nbw) q = k;  // no candidate (NaN input): no swap
            sym_swap(S, nsym, k, q, lane);
        }
        double gp;
        int r;
        {
            double v = (lane > k && lane < nbw) ? fabs(S.T[k * LDW + lane]) : -1.0;
            wave_argmax(v, lane, gp, r);
            if (!(gp > 0.0) || r <= k || r >= nbw) {
                gp = 0.0;
                r = -1;
            }
        }
        const double akk = fabs(S.T[k * LDW + k]);
        int two = 0, lifted = 0;
        double fkk_before = S.T[k * LDW + k];
        if (fmax(akk, gp) <= tiny) {
            lifted = 1;
        } else if (akk >= alpha * gp) {
            // 1x1 at k
        } else {
            double v2 = (lane >= k && lane < nbw && lane != r) ? fabs(S.T[r * LDW + lane]) : -1.0;
            double gr = wave_max(v2);
            if (gr < 0.0) gr = 0.0;
            if (akk * gr >= alpha * gp * gp) {
                // 1x1 at k
            } else if (fabs(S.T[r * LDW + r]) >= alpha * gr) {
                sym_swap(S, nsym, k, r, lane);
                fkk_before = S.T[k * LDW + k];
            } else {
                sym_swap(S, nsym, k + 1, r, lane);
                two = 1;
            }
        }
        if (two) {
            const double a = S.T[k * LDW + k] + S.sh[k];
            const double b = S.T[k * LDW + k + 1];
            const double c = S.T[(k + 1) * LDW + k + 1] + S.sh[k + 1];
            const double det = a * c - b * b;
            if (det == 0.0) {
                two = 0;
                fkk_before = S.T[k * LDW + k];
                lifted = 1;
            } else {
                // rows of the symmetric block below the pivot, and panel rows
                const bool act = lane >= k + 2 && lane < nsym;
                const double u0 = act ? S.T[k * LDW + lane] : 0.0;
                const double u1 = act ? S.T[(k + 1) * LDW + lane] : 0.0;
                const double l0 = act ? (u0 * c - u1 * b) / det : 0.0;
                const double l1 = act ? (u1 * a - u0 * b) / det : 0.0;
                if (lane < FM) {
                    S.w0[lane] = l0;
                    S.w1[lane] = l1;
                }
                __syncthreads();
                for (int j = k + 2; j < ncols; ++j) {
                    const double lj0 = S.w0[j], lj1 = S.w1[j];
                    if (act) S.T[j * LDW + lane] -= u0 * lj0 + u1 * lj1;
                }
                __syncthreads();
                if (act) {
                    S.T[k * LDW + lane] = l0;
                    S.T[(k + 1) * LDW + lane] = l1;
                }
                if (lane == 0) {
                    S.T[k * LDW + k + 1] = 0.0;
                    S.d[k] = a;
                    S.d[k + 1] = c;
                    S.doff[k] = b;
                    S.doff[k + 1] = 0.0;
                    S.pt[k] = 1;
                    S.pt[k + 1] = 2;
                    S.ed[k] = 0.0;
                    S.ed[k + 1] = 0.0;
                    S.fl[k] = 0;
                    S.fl[k + 1] = 0;
                    S.zs[k] = 0;
                    S.zs[k + 1] = 0;
                }
                __syncthreads();
                k += 2;
                continue;
            }
        }
        // 1x1 pivot at k
        if (lifted && lane == 0) S.T[k * LDW + k] = S.sg[k] * tiny;
        __syncthreads();
        double dk = S.T[k * LDW + k] + S.sh[k];  // static regularisation after the pivot
        const int sgk = S.sg[k];
        double q = -1.0;
        int zz = 0;
        if (lane > k && lane < nbw && S.sg[lane] == sgk) {
            double den = fabs(S.T[lane * LDW + lane] + S.sh[lane]);
            if (den == 0.0) zz = 1;
            else {
                double fjk = S.T[k * LDW + lane];
                q = fjk * fjk / den;
            }
        }
        double beta = wave_max(q);
        if (beta < 0.0) beta = 0.0;
        const int nz = wave_sum(zz);
        int flag = lifted ? PF_LIFT : 0;
        if (fabs(dk) < beta) {  // Proposition 3
            dk = sgk * beta;
            flag |= PF_PROP3;
        }
        if (!((sgk > 0 && dk > 0) || (sgk < 0 && dk < 0))) {  // keep the sign
            double mag = fabs(dk);
            if (beta > mag) mag = beta;
            if (tiny > mag) mag = tiny;
            dk = sgk * mag;
            flag |= PF_SIGN;
        }
        const double e = dk - (fkk_before + S.sh[k]);
        const bool act = lane > k && lane < nsym;
        const double li = act ? S.T[k * LDW + lane] / dk : 0.0;
        if (lane < FM) S.w0[lane] = (lane > k && lane < ncols) ? S.T[k * LDW + lane] : 0.0;  // column k
        __syncthreads();
        rank1_rows(S, k + 1, ncols, li, lane);
        __syncthreads();
        if (act) S.T[k * LDW + lane] = li;
        if (lane == 0) {
            S.d[k] = dk;
            S.doff[k] = 0.0;
            S.pt[k] = 0;
            S.ed[k] = e;
            S.fl[k] = flag;
            S.zs[k] = nz;
        }
        __syncthreads();
        k += 1;
    }
}

template <int FM>
__device__ inline void init_signs(PivShared<FM>& S, const DevPlan& D, const int32_t* rows, int fr, int sys,
                                  int lane) {
    const double rho = D.rho_sys[sys], delta = D.delta_sys[sys];
    if (lane < fr) {
        const bool pr = D.primal_new[rows[lane]] != 0;
        S.sg[lane] = pr ? -1 : 1;
        S.sh[lane] = pr ? -rho : delta;
        S.pm[lane] = lane;
    }
}

template <int FM>
__device__ inline void store_pivots(const PivShared<FM>& S, const DevPlan& D, int pos0, int k0, int nbw,
                                    int lane) {
    if (lane < nbw) {
        const int g = pos0 + lane;
        D.dval[g] = S.d[lane];
        D.doff[g] = S.doff[lane];
        D.ptype[g] = (int8_t)S.pt[lane];
        D.edyn[g] = S.ed[lane];
        D.pflag[g] = (uint8_t)S.fl[lane];
        D.zskip[g] = S.zs[lane];
        D.lperm[g] = k0 + S.pm[lane];
        D.lpinv[pos0 + S.pm[lane]] = k0 + lane;  // pos0 = c0 + k0
    }
}

// ---------------------------------------------------------------- factorisation kernels

// Small fronts (f <= FM <= 64): assembly of original entries and children's contribution blocks
// straight into LDS, then the whole partial factorisation there.
// A factor kernel launched for the FP64 redo of some systems skips the other systems' supernodes.
__device__ inline bool gated_off(const DevPlan& D, int s) { return D.gate && !D.gate[D.sn_sys[s]]; }

template <int FM>
__global__ __launch_bounds__(64) void k_small(DevPlan D, const Task* tasks, int64_t t0, PivotParams pp) {
    __shared__ PivShared<FM> S;
    constexpr int LDW = PivShared<FM>::LDW;
    const int lane = threadIdx.x;
    const int s = tasks[t0 + blockIdx.x].s;
    if (gated_off(D, s)) return;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    double* F = D.front + D.sn_off[s];
    const int32_t* rows = D.rows + D.sn_rowptr[s];
    for (int idx = lane; idx < FM * LDW; idx += 64) S.T[idx] = 0.0;
    __syncthreads();
    {  // original entries of the pivot columns (row position, column position, value)
        const int64_t e0 = D.kcol_ptr[c0], e1 = D.kcol_ptr[c0 + p];
        for (int64_t e = e0 + lane; e < e1; e += 64) {
            const int r = D.kloc[e], c = D.kcl[e];
            const double v = D.kval[e];
            S.T[c * LDW + r] = v;
            S.T[r * LDW + c] = v;
        }
    }
    __syncthreads();
    for (int q = D.ch_ptr[s]; q < D.ch_ptr[s + 1]; ++q) {  // children in ascending order
        const int ch = D.ch[q];
        const int cp = D.sn_p[ch], cb = D.sn_f[ch] - cp, cld = D.sn_ld[ch];
        const double* CF = D.front + D.sn_off[ch] + cp + (int64_t)cp * cld;
        const int32_t* rel = D.rel + D.rel_ptr[ch];
        // the child's contribution block (cb <= 64), all of it in flight at once
        const int ntot = cb * cb;
        for (int i0 = 0; i0 < ntot; i0 += 64 * 8) {
            double v[8];
            int ia[8], ib[8];
#pragma unroll
            for (int q2 = 0; q2 < 8; ++q2) {
                const int idx = i0 + q2 * 64 + lane;
                const int b = idx / cb, a = idx - b * cb;
                ia[q2] = a;
                ib[q2] = b;
                v[q2] = (idx < ntot && a >= b) ? CF[a + (int64_t)b * cld] : 0.0;
            }
#pragma unroll
            for (int q2 = 0; q2 < 8; ++q2) {
                const int idx = i0 + q2 * 64 + lane;
                if (idx < ntot && ia[q2] >= ib[q2]) {
                    const int ra = rel[ia[q2]], rb = rel[ib[q2]];
                    S.T[rb * LDW + ra] += v[q2];
                    if (ia[q2] != ib[q2]) S.T[ra * LDW + rb] += v[q2];
                }
            }
        }
        __syncthreads();
    }
    const int sys = D.sys_new[c0];
    init_signs(S, D, rows, f, sys, lane);
    __syncthreads();
    factor_window(S, f, p, D.knorm_sys[sys], pp, lane);
    for (int j = 0; j < f; ++j)
        if (lane >= j && lane < f) F[lane + (int64_t)j * ld] = S.T[j * LDW + lane];
    store_pivots(S, D, c0, 0, p, lane);
}

// readlane of a wave-uniform lane's 64-bit integer
__device__ inline int64_t readlane_i64(int64_t v, int l) {
    const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Large fronts: one workgroup per front column.  The column is summed in LDS from the
// original entries and, children in ascending order, the children's contribution-block
// columns that map onto it (the parent pulls; no atomics), then written once.  The list of
// (child, child column) pairs of each parent column is built by the analyse.
__global__ __launch_bounds__(256) void k_assemble(DevPlan D, const Task* tasks, int64_t t0) {
    extern __shared__ double buf[];
    const Task t = tasks[t0 + blockIdx.x];
    if (gated_off(D, t.s)) return;
    const int s = t.s, j = t.k0;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int nr = f - j;
    const int tid = threadIdx.x;
    for (int i = tid; i < nr; i += 256) buf[i] = 0.0;
    __syncthreads();
    if (j < p) {
        const int64_t e1 = D.kcol_ptr[c0 + j + 1];
        for (int64_t e = D.kcol_ptr[c0 + j] + tid; e < e1; e += 256) buf[D.kloc[e] - j] = D.kval[e];
    }
    __syncthreads();
    // the children's descriptions, 64 at a time (every wave loads the same: lane i those of
    // child q0 + i) and read by readlane, so a child costs one load latency, not three
    const int lane = tid & 63;
    for (int q0 = t.a; q0 < t.a + t.b; q0 += 64) {
    const int nq = min(64, t.a + t.b - q0);
    int m_lo = 0, m_cb = 0;
    int64_t m_rel = 0, m_col = 0;
    if (lane < nq) {
        const int ch = D.asm_child[q0 + lane];
        const int cp = D.sn_p[ch];
        m_lo = D.asm_col[q0 + lane];
        m_cb = D.sn_f[ch] - cp;
        m_rel = D.rel_ptr[ch];
        m_col = D.sn_off[ch] + (int64_t)(cp + m_lo) * D.sn_ld[ch] + cp;
    }
    for (int k = 0; k < nq; ++k) {
        const int lo = __builtin_amdgcn_readlane(m_lo, k), cb = __builtin_amdgcn_readlane(m_cb, k);
        const int32_t* rel = D.rel + readlane_i64(m_rel, k);
        const double* col = D.front + readlane_i64(m_col, k);
        // four entries' loads in flight per thread; the rows are distinct, so the order of the
        // additions into buf is that of the children alone
        for (int a = lo + tid; a < cb; a += 1024) {
            double v[4];
            int r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int x = a + 256 * u;
                v[u] = x < cb ? col[x] : 0.0;
                r[u] = x < cb ? rel[x] : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (r[u] >= 0) buf[r[u] - j] += v[u];
        }
        __syncthreads();
    }
    }
    double* out = D.front + D.sn_off[s] + (int64_t)j * ld + j;
    for (int i = tid; i < nr; i += 256) out[i] = buf[i];
}

// The same assembly with one wavefront per front column (four columns per workgroup), for
// levels whose fronts are at most 512 rows: many more columns in flight at once.  Each wave
// sums its column in its own LDS buffer; LDS operations of one wave complete in order, so
// the children's contributions are added in ascending child order without barriers.
__global__ __launch_bounds__(256) void k_assemble_w(DevPlan D, const Task* tasks, int64_t t0, int64_t ntask,
                                                    int maxf) {
    extern __shared__ double wbuf[];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t ti = (int64_t)blockIdx.x * 4 + wv;
    if (ti >= ntask) return;
    double* buf = wbuf + (int64_t)wv * maxf;
    const Task t = tasks[t0 + ti];
    const int s = t.s, j = t.k0;
    if (gated_off(D, s)) return;  // one task per wave, no barriers below
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int nr = f - j;
    for (int i = lane; i < nr; i += 64) buf[i] = 0.0;
    if (j < p) {
        const int64_t e1 = D.kcol_ptr[c0 + j + 1];
        for (int64_t e = D.kcol_ptr[c0 + j] + lane; e < e1; e += 64) buf[D.kloc[e] - j] = D.kval[e];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    // the children's descriptions, 64 at a time: lane i loads those of child q0 + i, and the
    // loop below reads them with readlane, so a child costs one load latency (its rows and
    // values), not three dependent ones
    for (int q0 = t.a; q0 < t.a + t.b; q0 += 64) {
    const int nq = min(64, t.a + t.b - q0);
    int m_lo = 0, m_cb = 0;
    int64_t m_rel = 0, m_col = 0;
    if (lane < nq) {
        const int ch = D.asm_child[q0 + lane];
        const int cp = D.sn_p[ch];
        m_lo = D.asm_col[q0 + lane];
        m_cb = D.sn_f[ch] - cp;
        m_rel = D.rel_ptr[ch];
        m_col = D.sn_off[ch] + (int64_t)(cp + m_lo) * D.sn_ld[ch] + cp;
    }
    for (int k = 0; k < nq; ++k) {
        const int lo = __builtin_amdgcn_readlane(m_lo, k), cb = __builtin_amdgcn_readlane(m_cb, k);
        const int32_t* rel = D.rel + readlane_i64(m_rel, k);
        const double* col = D.front + readlane_i64(m_col, k);
        for (int a0 = lo; a0 < cb; a0 += 256) {  // four rows per lane and trip, loads in flight together
            int ra[4];
            double va[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int a = a0 + 64 * u + lane;
                ra[u] = a < cb ? rel[a] - j : -1;
                va[u] = a < cb ? col[a] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (ra[u] >= 0) buf[ra[u]] += va[u];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    }
    double* out = D.front + D.sn_off[s] + (int64_t)j * ld + j;
    for (int i = lane; i < nr; i += 64) out[i] = buf[i];
}

// Helpers of the register-tiled window kernel.  readlane with a wave-uniform index.
__device__ inline double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// A value equal in every lane (an LDS read at a wave-uniform address) as a wave-uniform one.
__device__ inline double readfirst_d(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ inline double shfl_d(double v, int src) {  // value of lane src (ds_bpermute)
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Wave maximum of an unsigned 32-bit value (DPP rows then row broadcasts; lanes without a
// source contribute 0), read back from lane 63.
__device__ inline unsigned wave_umax(unsigned v) {
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Wave maxima of two unsigned values at once: the two DPP chains are interleaved, so each
// step of one hides the latency of the other.
__device__ inline void wave_umax2(unsigned& a, unsigned& b) {
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x111, 0xf, 0xf, false));
    b = max(b, (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, 0x111, 0xf, 0xf, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x112, 0xf, 0xf, false));
    b = max(b, (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, 0x112, 0xf, 0xf, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x114, 0xf, 0xf, false));
    b = max(b, (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, 0x114, 0xf, 0xf, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x118, 0xf, 0xf, false));
    b = max(b, (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, 0x118, 0xf, 0xf, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x142, 0xa, 0xf, false));
    b = max(b, (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, 0x142, 0xa, 0xf, false));
    a = max(a, (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, 0x143, 0xc, 0xf, false));
    b = max(b, (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, 0x143, 0xc, 0xf, false));
    a = (unsigned)__builtin_amdgcn_readlane((int)a, 63);
    b = (unsigned)__builtin_amdgcn_readlane((int)b, 63);
}

// Lanes where p holds, as a 64-bit mask (the builtin keeps it in scalar registers).
__device__ inline unsigned long long ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Ordering key of x >= 0 on the lanes with ok set: a non-negative double orders like its bit
// pattern read as an unsigned integer; bits + 1, so that 0 marks a lane without a candidate
// (or with NaN).
__device__ inline unsigned long long nn_key(double x, bool ok) {
    return (ok && x == x) ? (unsigned long long)__double_as_longlong(x) + 1ull : 0ull;
}

// Argmax of x >= 0 over the lanes with ok set (lowest lane on ties); -1 when no lane has a
// candidate.  The maximum of the 64-bit keys is taken on the upper halves first; the lower
// halves are compared only when several lanes share the largest upper half.
__device__ inline int wave_argmax_nn(double x, bool ok) {
    const unsigned long long key = nn_key(x, ok);
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned mh = wave_umax(hi);
    const unsigned long long m1 = ballot64(key != 0ull && hi == mh);
    if (m1 == 0ull) return -1;
    if ((m1 & (m1 - 1ull)) == 0ull) return __ffsll((long long)m1) - 1;
    const unsigned ml = wave_umax(hi == mh ? lo : 0u);
    return __ffsll((long long)ballot64(key != 0ull && hi == mh && lo == ml)) - 1;
}

// The rest of wave_argmax_nn once mh = wave_umax(upper half of key) is known (the reduction
// can then be issued early and the selection finished later).
__device__ inline int wave_argmax_finish(unsigned long long key, unsigned mh) {
    const unsigned hi = (unsigned)(key >> 32), lo = (unsigned)key;
    const unsigned long long m1 = ballot64(key != 0ull && hi == mh);
    if (m1 == 0ull) return -1;
    if ((m1 & (m1 - 1ull)) == 0ull) return __ffsll((long long)m1) - 1;
    const unsigned ml = wave_umax(hi == mh ? lo : 0u);
    return __ffsll((long long)ballot64(key != 0ull && hi == mh && lo == ml)) - 1;
}

// In one interleaved pass: the argmax r of x >= 0 over the okx lanes (lowest lane on ties,
// -1 if none) with its value xm, and the maximum ym of y >= 0 over the oky lanes (0 if none).
__device__ inline void wave_argmax_max_nn(double x, bool okx, double y, bool oky, int& r, double& xm,
                                          double& ym) {
    const unsigned long long kx = nn_key(x, okx), ky = nn_key(y, oky);
    unsigned hx = (unsigned)(kx >> 32), hy = (unsigned)(ky >> 32);
    wave_umax2(hx, hy);
    {  // the usual case: at most one lane attains each largest upper half, whose key is the maximum
        const unsigned long long bx = ballot64(kx != 0ull && (unsigned)(kx >> 32) == hx);
        const unsigned long long by = ballot64(ky != 0ull && (unsigned)(ky >> 32) == hy);
        if ((bx & (bx - 1ull)) == 0ull && (by & (by - 1ull)) == 0ull) {
            r = bx ? __ffsll((long long)bx) - 1 : -1;
            xm = bx ? readlane_d(x, r) : 0.0;
            ym = by ? readlane_d(y, __ffsll((long long)by) - 1) : 0.0;
            return;
        }
    }
    unsigned lx = (unsigned)(kx >> 32) == hx ? (unsigned)kx : 0u;
    unsigned ly = (unsigned)(ky >> 32) == hy ? (unsigned)ky : 0u;
    wave_umax2(lx, ly);
    const unsigned long long mx = ((unsigned long long)hx << 32) | lx, my = ((unsigned long long)hy << 32) | ly;
    r = mx ? __ffsll((long long)ballot64(kx == mx)) - 1 : -1;
    xm = mx ? __longlong_as_double((long long)(mx - 1ull)) : 0.0;
    ym = my ? __longlong_as_double((long long)(my - 1ull)) : 0.0;
}

// 1 / d to within about one unit in the last place: the hardware estimate refined by two
// Newton steps (fewer dependent operations than a correctly rounded division).  Where 1 / d
// overflows (|d| below about 2^-1024) the estimate's infinity is returned as it is.
__device__ inline double recip(double d) {
    const double r0 = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r0, 1.0);
    double r = fma(r0, e, r0);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return __builtin_isinf(r0) ? r0 : r;
}

// Exchange of the values held by lanes a and b (wave-uniform a, b).
__device__ inline int xchg_i(int v, int a, int b, int lane) {
    const int va = __builtin_amdgcn_readlane(v, a), vb = __builtin_amdgcn_readlane(v, b);
    return lane == a ? vb : (lane == b ? va : v);
}

__device__ inline double xchg_d(double v, int a, int b, int lane) {
    const double va = readlane_d(v, a), vb = readlane_d(v, b);
    return lane == a ? vb : (lane == b ? va : v);
}

// One pivot window [k0, k1) of a large front plus up to 64*NPG rows of the panel below it
// (chunk t.a), in one workgroup of four waves, one per SIMD.  Wave w holds window columns
// 16w .. 16w+15 of every row in registers: row group 0 is the window's own 64 rows, groups
// 1..NPG are panel rows; lane = row within a group.  Rows and columns never move: the
// symmetric interchanges of Section 4.5 are tracked as a position -> slot map, and every
// wave keeps, per position (= lane), the slot, its current diagonal, expected sign and
// static shift.  A pivot step costs one pivot-column broadcast through LDS (one barrier),
// wave-local DPP reductions for the tests (every wave takes the same decisions from the
// same data), and a rank-1 or rank-2 update of the register tile.  Every workgroup of the
// window repeats the identical decisions; the panel rows become L21.  Workgroup chunk 0
// also stores D, the pivot permutation and the factored block; the block goes to its upper
// triangle (transposed), because the other workgroups of this launch still read the
// unmodified lower part; k_finalize moves it.
template <int NPG>
__global__ __launch_bounds__(256) void k_window(DevPlan D, const Task* tasks, int64_t t0, PivotParams pp) {
    constexpr int RG = NPG + 1, NR = 64 * RG;
    __shared__ double colA[2][NR], colB[2][NR];
    __shared__ double Lb[64 * 64];  // L11: Lb[position * 64 + row slot]
    __shared__ int pinv_s[64];
    const int tid = threadIdx.x, lane = tid & 63, cq = tid >> 6;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, k0 = t.k0, chunk = t.a;
    if (gated_off(D, s)) return;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int k1 = min(k0 + NB, p), nbw = k1 - k0;
    double* F = D.front + D.sn_off[s];
    const int prow0 = k1 + 64 * NPG * chunk - 64 + lane;  // panel row of group g: prow0 + 64 g
    d16 T[RG];  // vector type: a wave-uniform element index becomes relative register addressing
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int c = 16 * cq + q;
        double v = 0.0;
        if (lane < nbw && c < nbw)  // lower triangle of the window block, mirrored
            v = lane >= c ? F[(k0 + lane) + (int64_t)(k0 + c) * ld] : F[(k0 + c) + (int64_t)(k0 + lane) * ld];
        T[0][q] = v;
    }
#pragma unroll
    for (int g = 1; g < RG; ++g) {
        const int pr = prow0 + 64 * g;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int c = 16 * cq + q;
            T[g][q] = (pr < f && c < nbw) ? F[pr + (int64_t)(k0 + c) * ld] : 0.0;
        }
    }
    // per position (= lane; initially position = slot): slot, diagonal, sign, static shift
    // The slot word packs the slot (bits 0-5) and whether its row is primal (bit 6), which
    // fixes the expected sign and the static shift; only the word and the diagonal move in an
    // interchange.
    int slotW = lane;
    double dgP = 0.0;
    const int sys = D.sys_new[c0];
    const double shPr = readfirst_d(-D.rho_sys[sys]), shDu = readfirst_d(D.delta_sys[sys]);
    if (lane < nbw) {
        dgP = F[(k0 + lane) + (int64_t)(k0 + lane) * ld];
        if (D.primal_new[D.rows[D.sn_rowptr[s] + k0 + lane]] != 0) slotW |= 64;
    }
    int slotP = slotW & 63, sgP = (slotW & 64) ? -1 : 1;
    double shP = (slotW & 64) ? shPr : shDu;
    auto derive = [&]() {
        slotP = slotW & 63;
        sgP = (slotW & 64) ? -1 : 1;
        shP = (slotW & 64) ? shPr : shDu;
    };
    // delta * ||M||_1 of the lift test; wave-uniform, so that every decision below, and the
    // pivot counter, stay scalar
    const double tiny = readfirst_d(pp.eps_lift * D.knorm_sys[sys]);
    const double alpha = pp.alpha;
    uint64_t elim = 0;  // eliminated slots
    double o_d = 0.0, o_off = 0.0, o_ed = 0.0;  // outputs of position = lane
    int o_pt = 0, o_fl = 0, o_zs = 0;
    int par = 0;
    int k = 0;
    // presort (largest |diagonal| of the window to position kk), done for pivot k + 1 (or k + 2)
    // at the end of the step of pivot k, as soon as the diagonal is updated
    auto presort_at = [&](int kk, int q) {
        q = (q < kk || q >= nbw) ? kk : q;  // no candidate (NaN input): no swap
        // exchanging position kk with itself changes nothing: no branch needed
        slotW = xchg_i(slotW, kk, q, lane);
        dgP = xchg_d(dgP, kk, q, lane);
        derive();
    };
    if (pp.presort && nbw > 0) presort_at(0, wave_argmax_nn(fabs(dgP), lane < nbw));
    while (k < nbw) {
        const int sk = __builtin_amdgcn_readlane(slotP, k);
        if (cq == (sk >> 4)) {
#pragma unroll
            for (int g = 0; g < RG; ++g) colA[par][64 * g + lane] = T[g][sk & 15];
        }
        // what the tests below need apart from the pivot column, before the barrier
        const double fkk = readlane_d(dgP, k);
        const int sgk0 = __builtin_amdgcn_readlane(sgP, k);
        const bool below = lane > k && lane < nbw;
        const double den = fabs(dgP + shP);
        const bool same = below && sgP == sgk0;
        const double rden = recip(den);
        __syncthreads();
        // gamma_p (largest |F_ik| below k in the window) and, for a 1x1 pivot on this column,
        // the Proposition 3 bound over same-sign positions, in one pass
        const double cP = colA[par][slotP];

        double gp, beta;
        int r, nz;
        {
            const double qv = (same && den != 0.0) ? cP * cP * rden : 0.0;
            wave_argmax_max_nn(fabs(cP), below, qv, same && den != 0.0, r, gp, beta);
            nz = __popcll(ballot64(same && den == 0.0));
            if (!(gp > 0.0)) {
                gp = 0.0;
                r = -1;
            }
        }
        const double akk = fabs(fkk);
        // the common outcomes (a lifted or an accepted 1x1 pivot at k) in one test
        const bool lift0 = fmax(akk, gp) <= tiny;
        const bool easy = lift0 | (akk >= alpha * gp);
        int piv = sk, two = 0, lifted = lift0, useB = 0;
        double fkk_before = fkk;
        if (!easy) {
            const int sr = __builtin_amdgcn_readlane(slotP, r);
            if (cq == (sr >> 4)) {
#pragma unroll
                for (int g = 0; g < RG; ++g) colB[par][64 * g + lane] = T[g][sr & 15];
            }
            __syncthreads();
            const double cB = colB[par][slotP];
            const int rl = wave_argmax_nn(fabs(cB), lane >= k && lane < nbw && lane != r);
            const double gr = rl >= 0 ? fabs(readlane_d(cB, rl)) : 0.0;
            const double frr = readlane_d(dgP, r);
            if (akk * gr >= alpha * gp * gp) {
                // 1x1 at k
            } else if (fabs(frr) >= alpha * gr) {
                slotW = xchg_i(slotW, k, r, lane);
                dgP = xchg_d(dgP, k, r, lane);
                derive();
                piv = sr;
                useB = 1;
                fkk_before = frr;
                // the Proposition 3 bound of the new pivot column
                const double cN = colB[par][slotP];
                const double den = fabs(dgP + shP);
                const bool same = lane > k && lane < nbw && sgP == __builtin_amdgcn_readlane(sgP, k);
                const double qn = (same && den != 0.0) ? cN * cN * recip(den) : 0.0;
                const int bl = wave_argmax_nn(qn, same && den != 0.0);
                beta = bl >= 0 ? readlane_d(qn, bl) : 0.0;
                nz = __popcll(ballot64(same && den == 0.0));
            } else {
                slotW = xchg_i(slotW, k + 1, r, lane);
                dgP = xchg_d(dgP, k + 1, r, lane);
                derive();
                two = 1;
            }
        }
        if (two) {
            const int sa = sk, sb = __builtin_amdgcn_readlane(slotP, k + 1);
            const double a = fkk + readlane_d(shP, k);
            const double b = readfirst_d(colA[par][sb]);  // same in every lane: keeps k wave-uniform
            const double c = readlane_d(dgP, k + 1) + readlane_d(shP, k + 1);
            const double det = a * c - b * b;
            if (det == 0.0) {
                two = 0;
                lifted = 1;
                piv = sk;
                fkk_before = fkk;
                // positions k+1 and r were exchanged: the bound over the new arrangement
                const double cN = colA[par][slotP];
                const double den = fabs(dgP + shP);
                const bool same = lane > k && lane < nbw && sgP == sgk0;
                const double qn = (same && den != 0.0) ? cN * cN * recip(den) : 0.0;
                const int bl = wave_argmax_nn(qn, same && den != 0.0);
                beta = bl >= 0 ? readlane_d(qn, bl) : 0.0;
                nz = __popcll(ballot64(same && den == 0.0));
            } else {
                elim |= (1ull << sa) | (1ull << sb);
                // multipliers of the columns (lane = slot), identical in every wave
                const bool crem = lane < nbw && !((elim >> lane) & 1);
                const double cu0 = colA[par][lane], cu1 = colB[par][lane];
                const double cl0 = crem ? (cu0 * c - cu1 * b) / det : 0.0;
                const double cl1 = crem ? (cu1 * a - cu0 * b) / det : 0.0;
                double lj0[16], lj1[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    lj0[q] = shfl_d(cl0, 16 * cq + q);
                    lj1[q] = shfl_d(cl1, 16 * cq + q);
                }
#pragma unroll
                for (int g = 0; g < RG; ++g) {
                    const bool rem = g > 0 ? prow0 + 64 * g < f : crem;
                    const double u0 = colA[par][64 * g + lane], u1 = colB[par][64 * g + lane];
                    const double l0 = rem ? (u0 * c - u1 * b) / det : 0.0;
                    const double l1 = rem ? (u1 * a - u0 * b) / det : 0.0;
#pragma unroll
                    for (int q = 0; q < 16; ++q) T[g][q] -= u0 * lj0[q] + u1 * lj1[q];
                    if (cq == 0) {
                        if (g == 0) {
                            Lb[k * 64 + lane] = l0;
                            Lb[(k + 1) * 64 + lane] = l1;
                        } else if (rem) {
                            F[prow0 + 64 * g + (int64_t)(k0 + k) * ld] = l0;
                            F[prow0 + 64 * g + (int64_t)(k0 + k + 1) * ld] = l1;
                        }
                    }
                }
                {  // diagonal of the remaining positions
                    const double pu0 = colA[par][slotP], pu1 = colB[par][slotP];
                    if (lane > k + 1 && lane < nbw)
                        dgP -= pu0 * ((pu0 * c - pu1 * b) / det) + pu1 * ((pu1 * a - pu0 * b) / det);
                }
                if (lane == k) {
                    o_d = a;
                    o_off = b;
                    o_pt = 1;
                    o_ed = 0.0;
                    o_fl = 0;
                    o_zs = 0;
                } else if (lane == k + 1) {
                    o_d = c;
                    o_off = 0.0;
                    o_pt = 2;
                    o_ed = 0.0;
                    o_fl = 0;
                    o_zs = 0;
                }
                if (pp.presort && k + 2 < nbw) presort_at(k + 2, wave_argmax_nn(fabs(dgP), lane > k + 1 && lane < nbw));
                par ^= 1;
                k += 2;
                continue;
            }
        }
        // 1x1 pivot at position k on slot piv
        const double(*colP) = useB ? colB[par] : colA[par];
        const int sgk = __builtin_amdgcn_readlane(sgP, k);
        const double shk = readlane_d(shP, k);
        // selects rather than branches: the values are wave-uniform
        const double fk = lifted ? sgk * tiny : fkk_before;
        double dk = fk + shk;  // static regularisation after the pivot
        const bool p3 = fabs(dk) < beta;  // Proposition 3
        dk = p3 ? sgk * beta : dk;
        const bool bad = !((sgk > 0 && dk > 0) || (sgk < 0 && dk < 0));  // keep the sign
        double mag = fabs(dk);
        mag = beta > mag ? beta : mag;
        mag = tiny > mag ? tiny : mag;
        dk = bad ? sgk * mag : dk;
        const int flag = (lifted ? PF_LIFT : 0) | (p3 ? PF_PROP3 : 0) | (bad ? PF_SIGN : 0);
        const double e = dk - (fkk_before + shk);
        elim |= 1ull << piv;
        const double rdk = recip(dk);
        double wq[16], lin[RG];
#pragma unroll
        for (int q = 0; q < 16; ++q) wq[q] = colP[16 * cq + q];
#pragma unroll
        for (int g = 0; g < RG; ++g) lin[g] = colP[64 * g + lane];
        {  // diagonal of the remaining positions, first: the next presort needs it
            const double cw = colP[slotP];
            dgP = (lane > k && lane < nbw) ? dgP - (cw * rdk) * cw : dgP;
        }
        if (lane == k) {
            o_d = dk;
            o_off = 0.0;
            o_pt = 0;
            o_ed = e;
            o_fl = flag;
            o_zs = nz;
        }
        // the wave maximum for the next presort is issued before the trailing update, so that
        // its dependent steps and the update's independent multiply-adds overlap
        const bool pnext = pp.presort && k + 1 < nbw;
        const unsigned long long nkey = nn_key(fabs(dgP), pnext && lane > k && lane < nbw);
        const unsigned nmh = wave_umax((unsigned)(nkey >> 32));
        {
            const bool crem = lane < nbw && !((elim >> lane) & 1);
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const bool rem = g > 0 ? prow0 + 64 * g < f : crem;
                const double li = rem ? lin[g] * rdk : 0.0;
#pragma unroll
                for (int q = 0; q < 16; ++q) T[g][q] -= li * wq[q];
                if (cq == 0) {
                    if (g == 0) Lb[k * 64 + lane] = li;
                    else if (rem) F[prow0 + 64 * g + (int64_t)(k0 + k) * ld] = li;
                }
            }
        }
        if (pnext) presort_at(k + 1, wave_argmax_finish(nkey, nmh));
        par ^= 1;
        k += 1;
    }
    if (cq == 0 && lane < nbw) pinv_s[slotP] = lane;
    __syncthreads();
    if (chunk == 0) {
        // L11 (strict lower, final order) transposed into the upper triangle: wave v takes
        // the columns (positions) v, v + 4, ...; lane = row slot
        const int pr = lane < nbw ? pinv_s[lane] : 0;
        for (int pc = cq; pc < nbw; pc += 4)
            if (lane < nbw && pr > pc) F[(k0 + pc) + (int64_t)(k0 + pr) * ld] = Lb[pc * 64 + lane];
        if (cq == 0 && lane < nbw) {
            const int g = c0 + k0 + lane;
            D.dval[g] = o_d;
            D.doff[g] = o_off;
            D.ptype[g] = (int8_t)o_pt;
            D.edyn[g] = o_ed;
            D.pflag[g] = (uint8_t)o_fl;
            D.zskip[g] = o_zs;
            D.lperm[g] = k0 + slotP;
            D.lpinv[c0 + k0 + slotP] = k0 + lane;
        }
    }
}

// Trailing update of one 64 x 64 lower tile: C -= L21 W^T with W = L21 D, on MFMA.
// The tile is computed transposed (C^T = W L21^T) so that each group of 16 lanes stores
// 16 consecutive rows of one column.  T = double: FP64 MFMA 16x16x4; T = float: operands
// rounded to FP32, FP32 MFMA with FP32 accumulation, result subtracted in FP64.
// Trailing updates stage the inner dimension in chunks of SYRK_CW columns (half a window):
// small LDS tiles and register arrays, so that three workgroups share a compute unit.
constexpr int SYRK_CW = 32;
constexpr int LDTG = SYRK_CW + 1;  // leading dimension of those LDS tiles, odd to spread banks

// One chunk of the inner dimension (columns kb .. kb + nbw) into registers: the L21 rows of
// the tile's row block (va) and column block (vc), all loads in flight at once.
__device__ inline void syrk_load_chunk(const double* F, int ld, int f, int cmax, int kb, int nbw, int R0, int C0,
                                       double* va, double* vc) {
    const int r = threadIdx.x & 63, kq = threadIdx.x >> 6;  // row r, columns kq, kq + 4, ...
#pragma unroll
    for (int t = 0; t < SYRK_CW / 4; ++t) {
        const int kk = kq + 4 * t;
        va[t] = (kk < nbw && R0 + r < f) ? F[R0 + r + (int64_t)(kb + kk) * ld] : 0.0;
        vc[t] = (kk < nbw && C0 + r < cmax) ? F[C0 + r + (int64_t)(kb + kk) * ld] : 0.0;
    }
}

// The chunk into LDS: As = L21 rows, Bs = W = L21 D on the column block (a 1x1 pivot scales
// its column, a 2x2 block mixes its two columns; the partner column is read again, 2x2 pivots
// are rare; the partner is read from the front, so a block across two chunks is fine).  dd,
// od, pt: D of the chunk's columns (od[-1] is the previous chunk's last column).
template <typename T>
__device__ inline void syrk_stage_chunk(const double* F, int ld, int cmax, int kb, int nbw, int C0,
                                        const double* va, const double* vc, const double* dd, const double* od,
                                        const int* pt, T* As, T* Bs) {
    const int r = threadIdx.x & 63, kq = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < SYRK_CW / 4; ++t) As[r * LDTG + kq + 4 * t] = (T)va[t];
    double wb[SYRK_CW / 4];
#pragma unroll
    for (int t = 0; t < SYRK_CW / 4; ++t) {
        const int kk = kq + 4 * t;
        double b = 0.0;
        if (kk < nbw && C0 + r < cmax) {
            const int ty = pt[kk];
            const double* cr = F + C0 + r + (int64_t)kb * ld;
            if (ty == 0) b = vc[t] * dd[kk];
            else if (ty == 1) b = vc[t] * dd[kk] + cr[(int64_t)(kk + 1) * ld] * od[kk];
            else b = cr[(int64_t)(kk - 1) * ld] * od[kk - 1] + vc[t] * dd[kk];
        }
        wb[t] = b;
    }
#pragma unroll
    for (int t = 0; t < SYRK_CW / 4; ++t) Bs[r * LDTG + kq + 4 * t] = (T)wb[t];
}

// C -= L21 W21^T on one 64 x 64 tile (rows R0.., columns C0.. below cmax, lower part) over the
// inner dimension in chunks of SYRK_CW columns (starting at column k0, nin columns in all).
// The products accumulate in the matrix cores (FP64) or are applied chunk by chunk (FP32), and
// C is read and written once.
template <typename T>
__device__ void syrk_tile(double* F, int ld, int f, int cmax, int k0, int nin, int R0, int C0,
                          const double* dd, const double* od, const int* pt, T* As, T* Bs) {
    const int tid = threadIdx.x;
    double va[SYRK_CW / 4], vc[SYRK_CW / 4];
    syrk_load_chunk(F, ld, f, cmax, k0, min(SYRK_CW, nin), R0, C0, va, vc);
    syrk_stage_chunk<T>(F, ld, cmax, k0, min(SYRK_CW, nin), C0, va, vc, dd, od, pt, As, Bs);
    const int wv = tid >> 6, l = tid & 63;
    const int wc = (wv >> 1) * 32, wr = (wv & 1) * 32;
    const int li = l & 15, lk = l >> 4;
    // this thread's 16 elements of the tile, loaded before the products so that their
    // latency overlaps them; element (i, j, v) at column C0 + wc + 16 i + cofs(v), row
    // R0 + wr + 16 j + li (f64 16x16x4 output: element (lk + 4v, li) of a 16 x 16 block;
    // f32 16x16x4 output: element (4 lk + v, li))
    double cv[2][2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = C0 + wc + i * 16 + (sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v);
                const int row = R0 + wr + j * 16 + li;
                cv[i][j][v] = (row < f && col < cmax && row >= col) ? F[row + (int64_t)col * ld] : 0.0;
            }
    using AccT = typename std::conditional<sizeof(T) == 8, d4, f4>::type;
    AccT acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = AccT{0, 0, 0, 0};
    const int nch = (nin + SYRK_CW - 1) / SYRK_CW;
    for (int c = 0; c < nch; ++c) {
        const int nbw = min(SYRK_CW, nin - SYRK_CW * c);
        const int kmax = (nbw + 3) & ~3;  // columns beyond the chunk are zero
        __syncthreads();
        for (int kk = 0; kk < kmax; kk += 4) {
            const T a0 = Bs[(wc + li) * LDTG + kk + lk];
            const T a1 = Bs[(wc + 16 + li) * LDTG + kk + lk];
            const T b0 = As[(wr + li) * LDTG + kk + lk];
            const T b1 = As[(wr + 16 + li) * LDTG + kk + lk];
            if constexpr (sizeof(T) == 8) {
                acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
            } else {
                acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
                acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
                acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
                acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
            }
        }
        if constexpr (sizeof(T) == 4) {
            // FP32 products are applied to the FP64 tile chunk by chunk, so that no more terms
            // are summed in FP32 than without grouping (one window)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) cv[i][j][v] -= (double)acc[i][j][v];
                    acc[i][j] = AccT{0, 0, 0, 0};
                }
        }
        if (c + 1 < nch) {
            const int kn = SYRK_CW * (c + 1), nn = min(SYRK_CW, nin - kn);
            syrk_load_chunk(F, ld, f, cmax, k0 + kn, nn, R0, C0, va, vc);
            __syncthreads();  // every wave has read this chunk from As and Bs
            syrk_stage_chunk<T>(F, ld, cmax, k0 + kn, nn, C0, va, vc, dd + kn, od + kn, pt + kn, As, Bs);
        }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = C0 + wc + i * 16 + (sizeof(T) == 8 ? lk + 4 * v : 4 * lk + v);
                const int row = R0 + wr + j * 16 + li;
                if (row < f && col < cmax && row >= col)
                    F[row + (int64_t)col * ld] = sizeof(T) == 4 ? cv[i][j][v] : cv[i][j][v] - (double)acc[i][j][v];
            }
}

// After all windows of a front: one task per (pivot window c, window w >= c).  w == c moves
// the window's factored diagonal block from the upper triangle into place; w > c permutes
// the rows of window w inside the 64 columns of window c as window w's pivot interchanges
// require.  Wave v handles columns 16v .. 16v+15, lane = row; each wave loads all of its
// values before it stores any, so no barrier is needed.
__device__ inline void finalize_task(const DevPlan& D, const Task t) {
    if (gated_off(D, t.s)) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int s = t.s, kc = t.k0, w = t.a;
    const int p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int ncol = min(NB, p - kc);
    double* F = D.front + D.sn_off[s];
    double v[16];
    if (w * NB == kc) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = 16 * wv + q;
            v[q] = (j < ncol && lane > j && lane < ncol) ? F[(kc + j) + (int64_t)(kc + lane) * ld] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = 16 * wv + q;
            if (j < ncol && lane > j && lane < ncol) F[(kc + lane) + (int64_t)(kc + j) * ld] = v[q];
        }
    } else {
        const int k0 = w * NB, nbw = min(NB, p - k0);
        const int src = lane < nbw ? D.lperm[c0 + k0 + lane] : 0;  // pre-pivot position now at k0 + lane
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = 16 * wv + q;
            v[q] = (j < ncol && lane < nbw) ? F[src + (int64_t)(kc + j) * ld] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int j = 16 * wv + q;
            if (j < ncol && lane < nbw) F[(k0 + lane) + (int64_t)(kc + j) * ld] = v[q];
        }
    }
}

// Tiles of the trailing update; workgroups past the first nsy take the level's finalize tasks
// from fin0 on (a launch may hold both: they touch disjoint parts of the fronts).
// Trailing-update tiles (lower 64 x 64 tiles of the trailing matrix): the task packs the inner
// range (one window, or several for a front with grouped windows) and whether only the next
// window's columns are updated.
__global__ __launch_bounds__(256, 3) void k_syrk(DevPlan D, const Task* tasks, int64_t t0, PivotParams pp,
                                                    int64_t nsy, int64_t fin0) {
    if ((int64_t)blockIdx.x >= nsy) {
        finalize_task(D, tasks[fin0 + (int64_t)blockIdx.x - nsy]);
        return;
    }
    __shared__ double As[64 * LDTG];
    __shared__ double Bs[64 * LDTG];
    __shared__ double dd[NB * SYRK_GROUP_MAX], od[NB * SYRK_GROUP_MAX];
    __shared__ int pt[NB * SYRK_GROUP_MAX];
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, k0 = t.k0 & SYRK_K0_MASK, cnt = ((t.k0 >> SYRK_COUNT_SHIFT) & 7) + 1;
    if (gated_off(D, s)) return;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int k1 = min(k0 + NB * cnt, p), nin = k1 - k0;
    // a narrow update stops at the end of the next window's columns
    const int cmax = (t.k0 & SYRK_NARROW) ? min(p, k1 + NB) : f;
    const int tid = threadIdx.x;
    for (int q = tid; q < NB * SYRK_GROUP_MAX; q += 256) {
        if (q < nin) {
            dd[q] = D.dval[c0 + k0 + q];
            od[q] = D.doff[c0 + k0 + q];
            pt[q] = D.ptype[c0 + k0 + q];
        } else {
            dd[q] = 0.0;
            od[q] = 0.0;
            pt[q] = 0;
        }
    }
    __syncthreads();
    double* F = D.front + D.sn_off[s];
    const int R0 = k1 + 64 * t.a, C0 = k1 + 64 * t.b;
    if (pp.mixed && f >= pp.f_mix)
        syrk_tile<float>(F, ld, f, cmax, k0, nin, R0, C0, dd, od, pt, (float*)As, (float*)Bs);
    else
        syrk_tile<double>(F, ld, f, cmax, k0, nin, R0, C0, dd, od, pt, As, Bs);
}

__global__ __launch_bounds__(256) void k_finalize(DevPlan D, const Task* tasks, int64_t t0) {
    finalize_task(D, tasks[t0 + blockIdx.x]);
}

// Trailing update of one 128 x 128 lower tile (full updates of large trailing matrices):
// C -= L21 W^T, W = L21 D.  Each wave owns a 64 x 64 quarter (4 x 4 MFMA blocks of 16 x 16),
// so every panel element read from LDS feeds 16 products and every panel byte fetched from L2
// feeds 16 flops (twice the 64 x 64 tile's).  The inner dimension goes through two LDS
// buffers in chunks of CW columns: while the matrix cores work on chunk c, the loads of chunk
// c + 1 are in flight, and they are written (with the D scaling) into the other buffer, one
// barrier per chunk.
//   T = double: FP64 MFMA 16x16x4, CW = 16, two workgroups per compute unit; C is read once
//   after the products and written once.
//   T = float (mixed precision): operands rounded to nearest into FP32, FP32 MFMA with FP32
//   accumulation over at most one pivot window (64 columns), then folded into FP64 copies of
//   the tile's entries held in registers, so that no more terms are summed in FP32 than in
//   one window; CW = 32, one workgroup per compute unit (the FP64 copies take 128 registers).
template <typename T, int CW>
__device__ void syrk128_tile(const DevPlan& D, const Task t, T* As, T* Bs, double* dd, double* od, int* pt) {
    constexpr int LDT = CW + 1;          // odd leading dimension spreads the LDS banks
    constexpr int HALF = CW / 2;         // columns of a chunk staged by one thread
    constexpr int BUF = 128 * LDT;       // one buffer of one panel
    const int s = t.s, k0 = t.k0 & SYRK_K0_MASK, cnt = ((t.k0 >> SYRK_COUNT_SHIFT) & 7) + 1;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int k1 = min(k0 + NB * cnt, p), nin = k1 - k0;
    const int tid = threadIdx.x;
    for (int q = tid; q < NB * SYRK_GROUP_MAX; q += 256) {
        const bool in = q < nin;
        dd[q] = in ? D.dval[c0 + k0 + q] : 0.0;
        od[q] = in ? D.doff[c0 + k0 + q] : 0.0;
        pt[q] = in ? (int)D.ptype[c0 + k0 + q] : 0;
    }
    double* F = D.front + D.sn_off[s];
    const int R0 = k1 + 128 * t.a, C0 = k1 + 128 * t.b;
    // staging: thread (r, h) moves row r of both panels, chunk columns HALF h .. HALF (h + 1) - 1
    const int r = tid & 127, h = tid >> 7;
    const bool rin = R0 + r < f, cin = C0 + r < f;
    const double* Ar = F + R0 + r;
    const double* Br = F + C0 + r;
    double va[HALF], vb[HALF];
    auto load = [&](int kb) {  // the chunk starting at inner column kb (relative to k0)
#pragma unroll
        for (int q = 0; q < HALF; ++q) {
            const int kk = kb + HALF * h + q;
            const bool ok = kk < nin;
            va[q] = (ok && rin) ? Ar[(int64_t)(k0 + kk) * ld] : 0.0;
            vb[q] = (ok && cin) ? Br[(int64_t)(k0 + kk) * ld] : 0.0;
        }
    };
    auto stage = [&](int kb, int buf) {
        T* Ab = As + buf * BUF;
        T* Bb = Bs + buf * BUF;
#pragma unroll
        for (int q = 0; q < HALF; ++q) {
            const int c = HALF * h + q, kk = kb + c;
            Ab[r * LDT + c] = (T)va[q];
            double w = 0.0;
            if (kk < nin && cin) {
                const int ty = pt[kk];
                if (ty == 0) w = vb[q] * dd[kk];
                else if (ty == 1) w = vb[q] * dd[kk] + Br[(int64_t)(k0 + kk + 1) * ld] * od[kk];
                else w = Br[(int64_t)(k0 + kk - 1) * ld] * od[kk - 1] + vb[q] * dd[kk];
            }
            Bb[r * LDT + c] = (T)w;
        }
    };
    const int wv = tid >> 6, l = tid & 63;
    const int wr = (wv & 1) * 64, wc = (wv >> 1) * 64;
    const int li = l & 15, lk = l >> 4;
    // a wave whose quarter lies above the diagonal of a diagonal tile has nothing to update
    const bool active = !(t.a == t.b && wr < wc);
    constexpr bool F64 = sizeof(T) == 8;
    using AccT = typename std::conditional<F64, d4, f4>::type;
    // element (i, j, v) of the quarter: column C0 + wc + 16 i + cofs(v), row R0 + wr + 16 j + li
    // (f64 16x16x4 output: element (lk + 4 v, li) of a block; f32 16x16x4: (4 lk + v, li))
    auto col_of = [&](int i, int v) { return C0 + wc + 16 * i + (F64 ? lk + 4 * v : 4 * lk + v); };
    auto row_of = [&](int j) { return R0 + wr + 16 * j + li; };
    AccT acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = AccT{0, 0, 0, 0};
    double cv[F64 ? 1 : 4][F64 ? 1 : 4][F64 ? 1 : 4];  // mixed: the FP64 tile entries
    if constexpr (!F64) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = col_of(i, v), row = row_of(j);
                    cv[i][j][v] = (active && row < f && col < f && row >= col) ? F[row + (int64_t)col * ld] : 0.0;
                }
    }
    load(0);
    __syncthreads();  // dd, od, pt
    stage(0, 0);
    __syncthreads();
    const int nch = (nin + CW - 1) / CW;
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) load(CW * (c + 1));
        if (active) {
            const T* Ab = As + buf * BUF;
            const T* Bb = Bs + buf * BUF;
#pragma unroll
            for (int kk = 0; kk < CW; kk += 4) {
                T a[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = Bb[(wc + 16 * i + li) * LDT + kk + lk];
#pragma unroll
                for (int j = 0; j < 4; ++j) b[j] = Ab[(wr + 16 * j + li) * LDT + kk + lk];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if constexpr (F64)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
                    }
            }
            if constexpr (!F64) {
                // a window's worth of FP32 products (or the task's last chunk) into FP64
                if (((c + 1) * CW) % NB == 0 || c + 1 == nch) {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) cv[i][j][v] -= (double)acc[i][j][v];
                            acc[i][j] = AccT{0, 0, 0, 0};
                        }
                }
            }
        }
        if (c + 1 < nch) stage(CW * (c + 1), buf ^ 1);
        __syncthreads();
    }
    if (!active) return;
    if constexpr (F64) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double cw[4][4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = col_of(i, v), row = row_of(j);
                    cw[j][v] = (row < f && col < f && row >= col) ? F[row + (int64_t)col * ld] : 0.0;
                }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = col_of(i, v), row = row_of(j);
                    if (row < f && col < f && row >= col) F[row + (int64_t)col * ld] = cw[j][v] - acc[i][j][v];
                }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int col = col_of(i, v), row = row_of(j);
                    if (row < f && col < f && row >= col) F[row + (int64_t)col * ld] = cv[i][j][v];
                }
    }
}

// 128 x 128 trailing-update tiles in FP64; workgroups past the first nsy take the level's
// finalize tasks from fin0 on (as in k_syrk).
constexpr int S128_CW64 = 16, S128_CW32 = 32;
__global__ __launch_bounds__(256, 2) void k_syrk128(DevPlan D, const Task* tasks, int64_t t0, int64_t nsy,
                                                    int64_t fin0) {
    if ((int64_t)blockIdx.x >= nsy) {
        finalize_task(D, tasks[fin0 + (int64_t)blockIdx.x - nsy]);
        return;
    }
    __shared__ double As[2 * 128 * (S128_CW64 + 1)];
    __shared__ double Bs[2 * 128 * (S128_CW64 + 1)];
    __shared__ double dd[NB * SYRK_GROUP_MAX], od[NB * SYRK_GROUP_MAX];
    __shared__ int pt[NB * SYRK_GROUP_MAX];
    if (gated_off(D, tasks[t0 + blockIdx.x].s)) return;
    syrk128_tile<double, S128_CW64>(D, tasks[t0 + blockIdx.x], As, Bs, dd, od, pt);
}

// The same tiles with FP32 products (mixed precision, fronts of order >= f_mix).
__global__ __launch_bounds__(256, 1) void k_syrk128f(DevPlan D, const Task* tasks, int64_t t0) {
    __shared__ float As[2 * 128 * (S128_CW32 + 1)];
    __shared__ float Bs[2 * 128 * (S128_CW32 + 1)];
    __shared__ double dd[NB * SYRK_GROUP_MAX], od[NB * SYRK_GROUP_MAX];
    __shared__ int pt[NB * SYRK_GROUP_MAX];
    if (gated_off(D, tasks[t0 + blockIdx.x].s)) return;
    syrk128_tile<float, S128_CW32>(D, tasks[t0 + blockIdx.x], As, Bs, dd, od, pt);
}

// ---------------------------------------------------------------- values of K

__global__ void k_init_scalars(DevPlan D, double rho, double delta, const double* rho_a, const double* delta_a) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) {
        D.sc->rho = rho;
        D.sc->delta = delta;
        D.sc->bad_theta = 0;
        D.sc->knorm = 0.0;
    }
    if (q < D.nsys) {
        D.rho_sys[q] = rho_a ? rho_a[q] : rho;
        D.delta_sys[q] = delta_a ? delta_a[q] : delta;
        D.knorm_sys[q] = 0.0;
    }
}

// Per-system shifts read from device arrays: a negative or non-finite rho or delta is reported
// as invalid input, as a Theta that is not positive and finite is.
__global__ void k_check_shifts(DevPlan D) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= D.nsys) return;
    const double r = D.rho_sys[q], d = D.delta_sys[q];
    if (!(r >= 0.0) || !(d >= 0.0) || !isfinite(r) || !isfinite(d)) atomicOr(&D.sc->bad_theta, 1);
}

// AS: dinv = 1/Theta (diagonal -(Theta^{-1}) of equation (augsys));
// NE: dinv = theta~ = 1/(1/Theta + rho) (equation (regul_matrix)).
__global__ void k_theta(DevPlan D, const double* theta) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.n) return;
    const double th = theta[j];
    if (!(th > 0.0) || !isfinite(th)) atomicOr(&D.sc->bad_theta, 1);
    if (D.mode == 1) D.dinv[j] = 1.0 / th;
    else D.dinv[j] = 1.0 / (1.0 / th + D.rho_sys[D.sys_col[j]]);
}

// Q_jj of a quadratic program (0 where Q has no diagonal entry)
__device__ inline double q_diag(const DevPlan& D, int j) { return D.qdiag[j] >= 0 ? D.qval[D.qdiag[j]] : 0.0; }

// Values of lower(K) in analyse order.  AS: A entries, the x diagonal -1/Theta_j (for a
// quadratic program -(1/Theta_j + Q_jj)), -Q_kj for Q's couplings, 0 on the y diagonal.
// NE: K_ik = sum_j (A_ij theta~_j) A_kj over the shared columns j in ascending order (fixed
// order, no atomics).
__global__ void k_values(DevPlan D, int64_t knnz) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= knnz) return;
    if (D.mode == 1) {
        const int64_t src = D.ksrc[e];
        double v;
        if (src >= 0) v = D.aval[src];
        else if (src == KSRC_ZERO) v = 0.0;
        else {
            const int64_t t = -1 - src;
            if (t >= D.n) v = -D.qval[t - D.n];
            else if (D.has_q) v = -(D.dinv[t] + q_diag(D, (int)t));
            else v = -D.dinv[t];
        }
        D.kval[e] = v;
    } else {
        double acc = 0.0;
        for (int64_t q = D.kpair_ptr[e]; q < D.kpair_ptr[e + 1]; ++q) {
            const int32_t a = D.kpair[2 * q], b = D.kpair[2 * q + 1];
            acc += (D.aval[a] * D.dinv[D.acol[a]]) * D.aval[b];
        }
        D.kval[e] = acc;
    }
}

// Row 1-norms of K_static in original numbering.
__global__ void k_rowsum(DevPlan D) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D.N) return;
    const int sys = D.sys_old[i];
    const double rho = D.rho_sys[sys], delta = D.delta_sys[sys];
    double s;
    if (D.mode == 1) {
        if (i < D.n) {
            if (D.has_q) s = fabs((D.dinv[i] + q_diag(D, i)) + rho) + D.qoff[i] + D.colabs[i];
            else s = (D.dinv[i] + rho) + D.colabs[i];
        } else {
            s = D.rowabs[i - D.n] + delta;
        }
    } else {
        s = 0.0;
        for (int64_t q = D.krs_ptr[i]; q < D.krs_ptr[i + 1]; ++q) {
            double v = D.kval[D.krs_ent[q]];
            if (D.krs_other[q] == i) v += delta;
            s += fabs(v);
        }
    }
    D.rowsum[i] = s;
}

// ||K_static||_1 of each system (one workgroup per system; K is symmetric, so the largest
// row sum).
__global__ __launch_bounds__(1024) void k_knorm(DevPlan D) {
    __shared__ double red[1024];
    const int q = blockIdx.x;
    const int64_t* rg = D.sys_rng + 4 * q;
    double m = 0.0;
#pragma unroll 8
    for (int64_t i = rg[0] + threadIdx.x; i < rg[1]; i += 1024) m = fmax(m, D.rowsum[i]);
#pragma unroll 8
    for (int64_t i = rg[2] + threadIdx.x; i < rg[3]; i += 1024) m = fmax(m, D.rowsum[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        D.knorm_sys[q] = red[0];
        if (D.nsys == 1) D.sc->knorm = red[0];
    }
}

// Sum over k != j of |Q_kj| per column of a quadratic program's Q (once per Q).
__global__ void k_hessian_norms(DevPlan D) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.n) return;
    double s = 0.0;
    for (int64_t e = D.qfcp[j]; e < D.qfcp[j + 1]; ++e)
        if (D.qfri[e] != j) s += fabs(D.qval[D.qfsrc[e]]);
    D.qoff[j] = s;
}

// Sum_i |A_ij| per column and sum_j |A_ij| per row (once per matrix).
__global__ void k_matrix_norms(DevPlan D) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < D.n) {
        double s = 0.0;
        for (int64_t e = D.acp[t]; e < D.acp[t + 1]; ++e) s += fabs(D.aval[e]);
        D.colabs[t] = s;
    }
    if (t < D.m) {
        double s = 0.0;
        for (int64_t q = D.arp[t]; q < D.arp[t + 1]; ++q) s += fabs(D.aval[D.are[q]]);
        D.rowabs[t] = s;
    }
}

// Inertia and regularisation counts over all pivot positions: per-block partials, then a
// fixed-order sum (k_factor_stats_final).  Partial q of block g: part[g * 10 + q], the eight
// counts (negative, positive, zero, 2x2, lifts, Proposition 3, sign rule, zero-skips), the
// largest |E_dyn| and whether some |E_dyn| exceeds tau_big ||K||_1.
constexpr int FS_PER_BLOCK = 512;

__global__ __launch_bounds__(256) void k_factor_stats(DevPlan D, PivotParams pp, double* part) {
    __shared__ double red[10][256];
    double c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double me = 0.0, big = 0.0;
    const int64_t k0 = (int64_t)blockIdx.x * FS_PER_BLOCK;
    const int64_t k1 = min((int64_t)D.N, k0 + FS_PER_BLOCK);
    for (int64_t k = k0 + threadIdx.x; k < k1; k += 256) {
        const double thr = pp.tau_big * D.knorm_sys[D.sys_new[k]];
        const int ty = D.ptype[k];
        if (ty == 0) {
            const double d = D.dval[k];
            if (d < 0) c[0] += 1;
            else if (d > 0) c[1] += 1;
            else c[2] += 1;
        } else if (ty == 1) {
            c[3] += 1;
            const double a = D.dval[k], b = D.doff[k], cc = D.dval[k + 1];
            const double det = a * cc - b * b;
            if (det < 0) { c[0] += 1; c[1] += 1; }
            else if (a + cc > 0) c[1] += 2;
            else c[0] += 2;
        }
        const uint8_t fl = D.pflag[k];
        c[4] += (fl & PF_LIFT) != 0;
        c[5] += (fl & PF_PROP3) != 0;
        c[6] += (fl & PF_SIGN) != 0;
        c[7] += D.zskip[k];
        const double e = fabs(D.edyn[k]);
        me = fmax(me, e);
        if (e > thr) big = 1.0;
    }
    for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = c[q];
    red[8][threadIdx.x] = me;
    red[9][threadIdx.x] = big;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
            for (int q = 8; q < 10; ++q) red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 10) part[blockIdx.x * 10 + threadIdx.x] = red[threadIdx.x][0];
}

// Combines the per-block partials: counts are integers held exactly in doubles and the others
// are maxima, so the result does not depend on the order of combination.
__global__ __launch_bounds__(64) void k_factor_stats_final(DevPlan D, const double* part, int nblk) {
    __shared__ double red[10][64];
    double t[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int g = threadIdx.x; g < nblk; g += 64) {
        for (int q = 0; q < 8; ++q) t[q] += part[g * 10 + q];
        for (int q = 8; q < 10; ++q) t[q] = fmax(t[q], part[g * 10 + q]);
    }
    for (int q = 0; q < 10; ++q) red[q][threadIdx.x] = t[q];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int q = 0; q < 10; ++q) t[q] = red[q][0];
    for (int g = 1; g < 64; ++g) {
        for (int q = 0; q < 8; ++q) t[q] += red[q][g];
        for (int q = 8; q < 10; ++q) t[q] = fmax(t[q], red[q][g]);
    }
    DevStats* st = D.st;
    st->nneg = (int64_t)t[0];
    st->npos = (int64_t)t[1];
    st->nzero = (int64_t)t[2];
    st->n2x2 = (int64_t)t[3];
    st->nlift = (int64_t)t[4];
    st->nprop3 = (int64_t)t[5];
    st->nsign = (int64_t)t[6];
    st->nzskip = (int64_t)t[7];
    st->max_edyn = t[8];
    st->large_reg = t[9] > 0;
    st->bad_theta = D.sc->bad_theta;
    if (D.nsys == 1) {  // a single system: its inertia is the total
        D.inertia_sys[0] = st->nneg;
        D.inertia_sys[1] = st->npos;
        D.inertia_sys[2] = st->nzero;
    }
}

// Inertia of each system from its own pivot positions (one workgroup per system).
__global__ __launch_bounds__(256) void k_sys_inertia(DevPlan D) {
    __shared__ int64_t red[3][256];
    const int q = blockIdx.x;
    int64_t c[3] = {0, 0, 0};
    for (int64_t t = D.sys_piv_ptr[q] + threadIdx.x; t < D.sys_piv_ptr[q + 1]; t += 256) {
        const int k = D.sys_piv[t];
        const int ty = D.ptype[k];
        if (ty == 0) {
            const double d = D.dval[k];
            c[d < 0 ? 0 : (d > 0 ? 1 : 2)]++;
        } else if (ty == 1) {
            const double a = D.dval[k], b = D.doff[k], cc = D.dval[k + 1];
            const double det = a * cc - b * b;
            if (det < 0) { c[0]++; c[1]++; }
            else if (a + cc > 0) c[1] += 2;
            else c[0] += 2;
        }
    }
    for (int v = 0; v < 3; ++v) red[v][threadIdx.x] = c[v];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int v = 0; v < 3; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) D.inertia_sys[3 * q + threadIdx.x] = red[threadIdx.x][0];
}

// Mixed precision: marks the systems whose factor broke down.  Level 1: a pivot that is not
// finite; 2: also a dynamic regularisation above tau_big ||K||_1 (a pivot whose computed
// value had to be replaced wholesale); 3: also any pivot that took Proposition 3 or the sign
// rule (an exact quasi-definite matrix needs neither, so the FP32 rounding of the Schur
// updates has changed that pivot's sign).  Block (c, q) scans chunk c of system q's pivot
// positions; redo is zero when the launch starts.
constexpr int MC_CHUNK = 4096;

__global__ __launch_bounds__(256) void k_mixed_check(DevPlan D, PivotParams pp) {
    const int q = blockIdx.y;
    const int64_t a = D.sys_piv_ptr[q] + (int64_t)blockIdx.x * MC_CHUNK;
    const int64_t b = min(D.sys_piv_ptr[q + 1], a + MC_CHUNK);
    const double big = pp.tau_big * D.knorm_sys[q];
    int bad = 0;
    for (int64_t t = a + threadIdx.x; t < b; t += 256) {
        const int k = D.sys_piv[t];
        bad |= !isfinite(D.dval[k]) || !isfinite(D.doff[k]) || !isfinite(D.edyn[k]);
        if (pp.mixed_check >= 2) bad |= fabs(D.edyn[k]) > big;
        if (pp.mixed_check >= 3) bad |= (D.pflag[k] & (PF_PROP3 | PF_SIGN)) != 0;
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(D.redo + q, 1);
}

__global__ __launch_bounds__(256) void k_mixed_count(DevPlan D) {
    __shared__ int red[256];
    int c = 0;
    for (int q = threadIdx.x; q < D.nsys; q += 256) c += D.redo[q];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) D.redo[D.nsys] = red[0];
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------- solve kernels

// Maximum that keeps a NaN: a residual or solution that is not finite must not report a small
// backward error.
__device__ inline double nmax(double a, double b) { return (a > b || a != a) ? a : b; }

__global__ void k_zero(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Right-hand side of the factorised system in original numbering:
// AS: [r7; r1];  NE: r8 = r1 + A theta~ r7 (equation (normeq)).
__global__ void k_rhs(DevPlan D, DevSolve S, const double* r7, const double* r1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N) return;
    double* b = S.b + (int64_t)r * D.N;
    if (D.mode == 1) {
        if (i < D.n) b[i] = r7 ? r7[i + (int64_t)r * D.n] : 0.0;
        else b[i] = r1[(i - D.n) + (int64_t)r * D.m];
    } else {
        double v = r1[i + (int64_t)r * D.m];
        if (r7)
            for (int64_t q = D.arp[i]; q < D.arp[i + 1]; ++q) {
                const int32_t e = D.are[q];
                const int32_t j = D.acol[e];
                v += D.aval[e] * (D.dinv[j] * r7[j + (int64_t)r * D.n]);
            }
        b[i] = v;
    }
}

__global__ void k_permute(DevPlan D, const double* src, double* xw, const int32_t* active) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= D.N || (active && !active[r])) return;
    xw[c + (int64_t)r * D.N] = src[D.perm[c] + (int64_t)r * D.N];
}

__global__ void k_unpermute(DevPlan D, const double* xw, double* dst, const int32_t* active) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= D.N || (active && !active[r])) return;
    dst[D.perm[c] + (int64_t)r * D.N] = xw[c + (int64_t)r * D.N];
}

// Solve kernels are instantiated per level with NBM >= the largest pivot block of the level
// (8, 16, 32 or 64), which sizes LDS tiles and register blocks; Lb holds a block with row
// stride NBM + 1: Lb[k * (NBM + 1) + i] = L(k0 + i, k0 + k), strictly lower, zero elsewhere.
template <int NBM>
struct BlockRegs {
    double v[(NBM * NBM + 255) / 256];
};

template <int NBM>
__device__ inline void load_block(BlockRegs<NBM>& b, const double* F, int ld, int k0, int nb, int tid) {
    constexpr int NT = (NBM * NBM + 255) / 256;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int idx = tid + 256 * t, i = idx % NBM, k = idx / NBM;
        b.v[t] = (idx < NBM * NBM && i < nb && k < nb && i > k) ? F[(k0 + i) + (int64_t)(k0 + k) * ld] : 0.0;
    }
}

template <int NBM>
__device__ inline void store_block(double* Lb, const BlockRegs<NBM>& b, int tid) {
    constexpr int LS = NBM + 1, NT = (NBM * NBM + 255) / 256;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int idx = tid + 256 * t;
        if (idx < NBM * NBM) Lb[(idx / NBM) * LS + idx % NBM] = b.v[t];
    }
}

template <int NBM>
__device__ inline void stage_block(double* Lb, const double* F, int ld, int k0, int nb, int tid) {
    BlockRegs<NBM> b;
    load_block<NBM>(b, F, ld, k0, nb, tid);
    store_block<NBM>(Lb, b, tid);
}

// The inverse of a unit lower diagonal block (nb x nb, column-major, unit diagonal stored)
// into the same LDS layout as stage_block: Lb[k * (NBM + 1) + i] = Linv(i, k).
template <int NBM>
__device__ inline void load_inv(BlockRegs<NBM>& b, const double* Li, int nb, int tid) {
    constexpr int NT = (NBM * NBM + 255) / 256;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int idx = tid + 256 * t, i = idx % NBM, k = idx / NBM;
        b.v[t] = (idx < NBM * NBM && i < nb && k < nb && i >= k) ? Li[i + (int64_t)k * nb] : 0.0;
    }
}

// y[0..nb) <- Linv y (forward) or Linv^T y (backward) with the inverse staged in Lb: every
// thread sums a fixed slice of k, the slices are added in a fixed order.  part: 256 doubles
// of LDS.  Ends with a barrier.
template <int NBM, bool TRANS>
__device__ inline void block_inv_apply(const double* Lb, double* y, int nb, double* part, int tid) {
    constexpr int LS = NBM + 1;
    constexpr int KC = NBM * NBM >= 256 ? NBM * NBM / 256 : 1, NP = NBM / KC;
    const int i = tid % NBM, q = tid / NBM;
    if (q < NP) {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int u = 0; u < KC; u += 2) {
            const int k = q * KC + u;
            if (k < nb) a0 += (TRANS ? Lb[i * LS + k] : Lb[k * LS + i]) * y[k];
            if (u + 1 < KC && k + 1 < nb) a1 += (TRANS ? Lb[i * LS + k + 1] : Lb[(k + 1) * LS + i]) * y[k + 1];
        }
        part[q * NBM + i] = a0 + a1;
    }
    __syncthreads();
    if (tid < nb) {
        double v = 0.0;
#pragma unroll
        for (int qq = 0; qq < NP; ++qq) v += part[qq * NBM + tid];
        y[tid] = v;
    }
    __syncthreads();
}

// Triangular solves on the staged block in one wavefront with the block in registers: lane
// i holds row i (forward) or column i (backward) and its y value; each step broadcasts one
// finished y by readlane.
template <int NBM>
__device__ inline double trsv_fwd_wave(const double* Lb, double y, int lane) {
    constexpr int LS = NBM + 1;
    double l[NBM];
#pragma unroll
    for (int k = 0; k < NBM; ++k) l[k] = lane < NBM ? Lb[k * LS + lane] : 0.0;
#pragma unroll
    for (int k = 0; k < NBM - 1; ++k) {
        const double z = readlane_d(y, k);
        if (lane > k) y -= l[k] * z;
    }
    return y;
}

template <int NBM>
__device__ inline double trsv_bwd_wave(const double* Lb, double y, int lane) {
    constexpr int LS = NBM + 1;
    double c[NBM];
#pragma unroll
    for (int i = 0; i < NBM; ++i) c[i] = lane < NBM ? Lb[lane * LS + i] : 0.0;
#pragma unroll
    for (int i = NBM - 1; i > 0; --i) {
        const double z = readlane_d(y, i);
        if (lane < i) y -= c[i] * z;
    }
    return y;
}

// Forward substitution with unit L and the D solve for one supernode.  The parent gathers
// its children's contribution vectors (ascending order, no atomics).  y: f doubles of LDS;
// Lb: 64 x 65 doubles of LDS holding the current 64 x 64 diagonal block of L.
template <int NBM>
__device__ void fwd_supernode(const DevPlan& D, const DevSolve& S, int s, const int32_t* active, double* y,
                              double* Lb, double* part) {
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const double* F = D.front + D.sn_off[s];
    const int tid = threadIdx.x;
    // Values that do not depend on the right-hand side, loaded before anything waits: the first
    // trip of rows below the first block (RT rows per thread), and D of pivot tid.
    // (with NBM = 64 the prefetched rows would not fit in registers beside the rest)
    constexpr int RT = NBM <= 32 ? 2 : 1;
    constexpr bool PF = NBM <= 32;
    const int k1f = min(64, p), nbf = k1f;
    double lr[RT][PF ? NBM : 1];
    if constexpr (PF) {
#pragma unroll
        for (int u = 0; u < RT; ++u) {
            const int i = k1f + tid + 256 * u;
#pragma unroll
            for (int k = 0; k < NBM; ++k) lr[u][k] = (i < f && k < nbf) ? F[i + (int64_t)k * ld] : 0.0;
        }
    }
    int d_ty = 0, d_perm = 0;
    double d_a = 1.0, d_b = 0.0, d_c = 1.0;
    if (tid < p) {
        d_ty = D.ptype[c0 + tid];
        d_perm = D.lperm[c0 + tid];
        const int k2 = d_ty == 2 ? tid - 1 : tid;
        d_a = D.dval[c0 + k2];
        d_b = d_ty ? D.doff[c0 + k2] : 0.0;
        d_c = d_ty ? D.dval[c0 + k2 + 1] : 1.0;
    }
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        double* xw = S.xw + (int64_t)r * D.N;
        // blocks of more than 8 pivots are solved with their precomputed inverse, smaller ones
        // by a serial sweep in one wavefront
        constexpr bool INV = NBM > 8;
        const double* Linv = INV ? D.linv + D.inv_off[s] : nullptr;
        BlockRegs<NBM> b0;  // the first diagonal block (or its inverse), loaded along with the gather
        if constexpr (INV) load_inv<NBM>(b0, Linv, min(64, p), tid);
        else load_block<NBM>(b0, F, ld, 0, min(64, p), tid);
        {  // front row t (pre-pivot numbering): own entry plus the children's contributions
           // in ascending child order; pivot rows moved in factorisation (lpinv).  Four rows
           // per thread and trip, so that their loads are in flight together.
            const int64_t* gp = D.fg_ptr + D.sn_rowptr[s];
            const double* ub = S.ub + (int64_t)r * D.ub_total;
            for (int tb = 0; tb < f; tb += 1024) {
                int64_t qa[4], qe[4];
                double v[4];
                int dst[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int t = tb + tid + 256 * u;
                    const bool on = t < f;
                    qa[u] = on ? gp[t] : 0;
                    qe[u] = on ? gp[t + 1] : 0;
                    v[u] = (on && t < p) ? xw[c0 + t] : 0.0;
                    dst[u] = on ? (t < p ? D.lpinv[c0 + t] : t) : -1;
                }
                // four contributions of each of the four rows per trip: their source indices,
                // then their values, in flight together (added in list order)
                bool more = true;
                while (more) {
                    int64_t src[4][4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int j = 0; j < 4; ++j) src[u][j] = qa[u] + j < qe[u] ? D.fg_src[qa[u] + j] : -1;
                    double val[4][4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int j = 0; j < 4; ++j) val[u][j] = src[u][j] >= 0 ? ub[src[u][j]] : 0.0;
                    more = false;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (src[u][j] >= 0) v[u] += val[u][j];
                        qa[u] += 4;
                        more |= qa[u] < qe[u];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (dst[u] >= 0) y[dst[u]] = v[u];
            }
        }
        store_block<NBM>(Lb, b0, tid);
        __syncthreads();
        for (int k0 = 0; k0 < p; k0 += 64) {
            const int k1 = min(k0 + 64, p), nb = k1 - k0;
            if (k0 > 0) {
                BlockRegs<NBM> bk;
                if constexpr (INV) load_inv<NBM>(bk, Linv + 4096 * (k0 / 64), nb, tid);
                else load_block<NBM>(bk, F, ld, k0, nb, tid);
                store_block<NBM>(Lb, bk, tid);
                __syncthreads();
            }
            if constexpr (INV) {
                block_inv_apply<NBM, false>(Lb, y + k0, nb, part, tid);  // y_b <- Linv y_b
            } else {
                if (tid < 64) {
                    const double y0 = tid < nb ? y[k0 + tid] : 0.0;
                    const double v = trsv_fwd_wave<NBM>(Lb, y0, tid);
                    if (tid < nb) y[k0 + tid] = v;
                }
                __syncthreads();
            }
            // rows below: RT rows per thread and trip, their loads in flight together; the
            // first block's first trip uses the rows loaded at the start
            for (int i = k1 + tid; i < f; i += 256 * RT) {
                double la[RT][NBM];
                if (PF && k0 == 0 && i == k1 + tid) {
#pragma unroll
                    for (int u = 0; u < RT; ++u)
#pragma unroll
                        for (int k = 0; k < NBM; ++k) la[u][k] = lr[u][PF ? k : 0];
                } else {
#pragma unroll
                    for (int u = 0; u < RT; ++u) {
                        const double* Li = F + i + 256 * u + (int64_t)k0 * ld;
                        const bool on = i + 256 * u < f;
#pragma unroll
                        for (int k = 0; k < NBM; ++k) la[u][k] = (on && k < nb) ? Li[(int64_t)k * ld] : 0.0;
                    }
                }
                double a0[RT], a1[RT];
#pragma unroll
                for (int u = 0; u < RT; ++u) a0[u] = a1[u] = 0.0;
#pragma unroll
                for (int k = 0; k < NBM; k += 2) {
                    const double y0 = k < nb ? y[k0 + k] : 0.0, y1 = k + 1 < nb ? y[k0 + k + 1] : 0.0;
#pragma unroll
                    for (int u = 0; u < RT; ++u) {
                        if (k < nb) a0[u] += la[u][k] * y0;
                        if (k + 1 < nb) a1[u] += la[u][k + 1] * y1;
                    }
                }
#pragma unroll
                for (int u = 0; u < RT; ++u)
                    if (i + 256 * u < f) y[i + 256 * u] -= a0[u] + a1[u];
            }
            __syncthreads();
        }
        double* u = S.ub + D.ub_off[s] + (int64_t)r * D.ub_total;
        for (int i = p + tid; i < f; i += 256) u[i - p] = y[i];
        for (int k = tid; k < p; k += 256) {  // block-diagonal D
            int ty, perm;
            double a, b, c;
            if (k == tid) {
                ty = d_ty, perm = d_perm, a = d_a, b = d_b, c = d_c;
            } else {
                ty = D.ptype[c0 + k];
                perm = D.lperm[c0 + k];
                const int k2 = ty == 2 ? k - 1 : k;
                a = D.dval[c0 + k2];
                b = ty ? D.doff[c0 + k2] : 0.0;
                c = ty ? D.dval[c0 + k2 + 1] : 1.0;
            }
            double v;
            if (ty == 0) v = y[k] / a;
            else if (ty == 1) v = (c * y[k] - b * y[k + 1]) / (a * c - b * b);
            else v = (a * y[k] - b * y[k - 1]) / (a * c - b * b);
            xw[c0 + perm] = v;
        }
        __syncthreads();
    }
}

// Backward substitution with L^T for one supernode (its ancestors are done).  part: 4 x 64
// doubles of LDS for the partial sums of the rows below each block; Lt: a 64 x 65 tile.
template <int NBM>
__device__ void bwd_supernode(const DevPlan& D, const DevSolve& S, int s, const int32_t* active, double* y,
                              double* Lb, double* part, double* Lt) {
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const double* F = D.front + D.sn_off[s];
    const int32_t* rows = D.rows + D.sn_rowptr[s];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        double* xw = S.xw + (int64_t)r * D.N;
        const int nblk = (p + 63) / 64;
        constexpr bool INV = NBM > 8;
        const double* Linv = INV ? D.linv + D.inv_off[s] : nullptr;
        BlockRegs<NBM> bl;  // the last diagonal block (or its inverse), loaded along with y
        if constexpr (INV) load_inv<NBM>(bl, Linv + 4096 * (nblk - 1), p - (nblk - 1) * 64, tid);
        else load_block<NBM>(bl, F, ld, (nblk - 1) * 64, p - (nblk - 1) * 64, tid);
        for (int ib = 0; ib < f; ib += 1024) {  // four rows per thread and trip
            int src[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int i = ib + tid + 256 * u;
                src[u] = i < p ? c0 + D.lperm[c0 + i] : (i < f ? rows[i] : -1);
            }
            double v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = src[u] >= 0 ? xw[src[u]] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (src[u] >= 0) y[ib + tid + 256 * u] = v[u];
        }
        store_block<NBM>(Lb, bl, tid);
        __syncthreads();
        for (int bk = nblk - 1; bk >= 0; --bk) {
            const int k0 = bk * 64, k1 = min(k0 + 64, p), nb = k1 - k0;
            if (bk < nblk - 1) {
                BlockRegs<NBM> bb;
                if constexpr (INV) load_inv<NBM>(bb, Linv + 4096 * bk, nb, tid);
                else load_block<NBM>(bb, F, ld, k0, nb, tid);
                store_block<NBM>(Lb, bb, tid);  // read only after the barriers below
            }
            {  // rows below the block, sum_i L(i, k) y_i: tiles of 64 rows loaded coalesced (lane =
               // row, wave wv takes columns wv, wv + 4, ...; the next tile in flight while the
               // current one is accumulated per lane), then one reduction over the lanes: column
               // c's four partial sums are its lanes 0-15, 16-31, 32-47 and 48-63, in order
                constexpr int NT = NBM / 4;
                double accv[NT], cur[NT], nxt[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) accv[t] = 0.0;
                auto load = [&](int i0, double* v) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        const int k = wv + 4 * t, i = i0 + lane;
                        v[t] = (k < nb && i < f) ? F[i + (int64_t)(k0 + k) * ld] : 0.0;
                    }
                };
                load(k1, cur);
                for (int i0 = k1; i0 < f; i0 += 64) {
                    if (i0 + 64 < f) load(i0 + 64, nxt);
                    const double yi = i0 + lane < f ? y[i0 + lane] : 0.0;
#pragma unroll
                    for (int t = 0; t < NT; ++t) accv[t] += cur[t] * yi;
#pragma unroll
                    for (int t = 0; t < NT; ++t) cur[t] = nxt[t];
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) Lt[(wv + 4 * t) * 65 + lane] = accv[t];
                __syncthreads();
                const int c = tid & 63;
                double sq = 0.0;
                if (c < NBM) {
#pragma unroll
                    for (int j = 0; j < 16; ++j) sq += Lt[c * 65 + 16 * wv + j];
                }
                part[wv * 64 + c] = sq;
            }
            __syncthreads();
            if constexpr (INV) {
                if (tid < nb) y[k0 + tid] -= ((part[tid] + part[64 + tid]) + part[128 + tid]) + part[192 + tid];
                __syncthreads();
                block_inv_apply<NBM, true>(Lb, y + k0, nb, part, tid);  // y_b <- Linv^T y_b
            } else {
                if (tid < 64) {
                    double v = 0.0;
                    if (tid < nb) v = y[k0 + tid] - (((part[tid] + part[64 + tid]) + part[128 + tid]) + part[192 + tid]);
                    v = trsv_bwd_wave<NBM>(Lb, v, tid);
                    if (tid < nb) y[k0 + tid] = v;
                }
                __syncthreads();
            }
        }
        for (int k = tid; k < p; k += 256) xw[c0 + D.lperm[c0 + k]] = y[k];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- big-supernode solves
// Supernodes with large fronts are solved by many workgroups, all right-hand sides at once,
// in the work space Y (rows of supernode s at Y + yoff[s], pivot rows in post-pivot order,
// right-hand side r at offset r * ytot).  A launch is one step for every big supernode of a
// tree level: gather, per 64-pivot block a diagonal solve and a row-chunk update, finish;
// backward: load, per block (last first) row-chunk partial sums and a diagonal solve, store.

__device__ inline bool big_inactive(const DevSolve& S, const int32_t* active) {
    if (!active) return false;
    for (int r = 0; r < S.nrhs; ++r)
        if (active[r]) return false;
    return true;
}

__global__ __launch_bounds__(256) void k_sgather(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                                 const int32_t* active) {
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, i = 256 * t.k0 + threadIdx.x;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s];
    if (i >= f) return;
    const int64_t* gp = D.fg_ptr + D.sn_rowptr[s];
    const int64_t q0 = gp[i], q1 = gp[i + 1];
    const int64_t dst = D.yoff[s] + (i < p ? D.lpinv[c0 + i] : i);
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        const double* xw = S.xw + (int64_t)r * D.N;
        const double* ub = S.ub + (int64_t)r * D.ub_total;
        double v = i < p ? xw[c0 + i] : 0.0;
        for (int64_t q = q0; q < q1; q += 4) {  // four contributions in flight, added in list order
            int64_t src[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) src[j] = q + j < q1 ? D.fg_src[q + j] : -1;
            double val[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) val[j] = src[j] >= 0 ? ub[src[j]] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (src[j] >= 0) v += val[j];
        }
        S.Y[dst + (int64_t)r * S.ytot] = v;
    }
}

// Big supernodes are solved in blocks of SB = 256 pivots: per block one launch of one workgroup
// per supernode (the block's diagonal solve: four 64-pivot sub-blocks in sequence, y kept in
// LDS) and one launch over the rows below (all 256 columns of the block at once), so that a
// pass takes two launches per 256 pivots.
constexpr int SB = SOLVE_BLOCK;
static_assert(SB == 256, "one row per thread of a 256-thread workgroup within a block");

// forward: y_J <- L_JJ^{-1} y_J for the block J of 256 pivots, right-hand sides eight at a
// time: per 64-pivot sub-block, its precomputed inverse applied by all 256 threads, then the
// update of the block's later rows
__global__ __launch_bounds__(256) void k_sfdiag(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                                const int32_t* active) {
    __shared__ double Lb[64 * 65];
    __shared__ double yb[SB * 8];
    __shared__ double part[256];
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, k0 = SB * t.k0;
    const int p = D.sn_p[s], ld = D.sn_ld[s];
    const int nbJ = min(SB, p - k0);
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const double* F = D.front + D.sn_off[s];
    double* Ys = S.Y + D.yoff[s] + k0;
    for (int rg = 0; rg < S.nrhs; rg += 8) {
        const int nr = min(8, S.nrhs - rg);
        for (int idx = tid; idx < SB * 8; idx += 256) {
            const int i = idx & (SB - 1), rr = idx / SB;
            yb[idx] = (i < nbJ && rr < nr) ? Ys[i + (int64_t)(rg + rr) * S.ytot] : 0.0;
        }
        for (int a = 0; 64 * a < nbJ; ++a) {
            const int nb = min(64, nbJ - 64 * a);
            __syncthreads();  // yb written; the previous sub-block's update is done with Lb
            {
                BlockRegs<64> b;
                load_inv<64>(b, D.linv + D.inv_off[s] + 4096 * (int64_t)(4 * t.k0 + a), nb, tid);
                store_block<64>(Lb, b, tid);
            }
            __syncthreads();
            for (int rr = 0; rr < nr; ++rr) {  // rr and active[] are the same for the workgroup
                if (active && !active[rg + rr]) continue;
                block_inv_apply<64, false>(Lb, yb + SB * rr + 64 * a, nb, part, tid);
            }
            __syncthreads();
            // the rest of the block: rows 64 (a + 1) .. nbJ, columns of sub-block a
            const int i = 64 * (a + 1) + tid;
            if (i < nbJ) {
                double l[64];
                const double* Li = F + k0 + i + (int64_t)(k0 + 64 * a) * ld;
#pragma unroll
                for (int k = 0; k < 64; ++k) l[k] = k < nb ? Li[(int64_t)k * ld] : 0.0;
                for (int rr = 0; rr < nr; ++rr) {
                    const double* yv = yb + SB * rr + 64 * a;
                    double a0 = 0.0, a1 = 0.0;
#pragma unroll
                    for (int k = 0; k < 64; k += 2) {
                        a0 += l[k] * yv[k];
                        a1 += l[k + 1] * yv[k + 1];
                    }
                    yb[SB * rr + i] -= a0 + a1;
                }
            }
        }
        __syncthreads();
        for (int idx = tid; idx < SB * 8; idx += 256) {
            const int i = idx & (SB - 1), rr = idx / SB;
            if (i < nbJ && rr < nr && (!active || active[rg + rr])) Ys[i + (int64_t)(rg + rr) * S.ytot] = yb[idx];
        }
        __syncthreads();
    }
}

// rows below block J: y_i -= sum_k L(i, k0 + k) y_{k0 + k} over the block's 256 columns.  One
// workgroup takes 64 rows of the task's 256-row chunk (blockIdx.y); wave q sums the block's
// columns 64q .. 64q+63 with that part of its row in registers (lane = row), and wave 0 adds
// the four partial sums in column order.  The block's y values pass through LDS sixteen
// right-hand sides at a time.
__global__ __launch_bounds__(256) void k_sfupd(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                               const int32_t* active) {
    __shared__ double Yb[SB * 16];
    __shared__ double part[4 * 16 * 64];
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, k0 = SB * t.k0;
    const int f = D.sn_f[s], p = D.sn_p[s], ld = D.sn_ld[s];
    const int k1 = min(k0 + SB, p), nbJ = k1 - k0;
    const int tid = threadIdx.x, q = tid >> 6, lane = tid & 63;
    double* Ys = S.Y + D.yoff[s];
    const int i = k1 + 256 * t.a + 64 * (int)blockIdx.y + lane;
    const int nb = min(64, nbJ - 64 * q);  // columns of this wave's sub-block (<= 0: none)
    const double* Li = D.front + D.sn_off[s] + min(i, f - 1) + (int64_t)(k0 + 64 * q) * ld;
    double l[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) l[k] = (k < nb && i < f) ? Li[(int64_t)k * ld] : 0.0;
    for (int rg = 0; rg < S.nrhs; rg += 16) {
        const int nr = min(16, S.nrhs - rg);
        __syncthreads();  // the previous group is done with Yb and part
        for (int idx = tid; idx < SB * 16; idx += 256) {
            const int k = idx & (SB - 1), rr = idx / SB;
            Yb[idx] = (k < nbJ && rr < nr) ? Ys[k0 + k + (int64_t)(rg + rr) * S.ytot] : 0.0;
        }
        __syncthreads();
        if (nb > 0) {
#pragma unroll
            for (int rr = 0; rr < 16; ++rr) {
                if (rr >= nr) break;
                const double* yb = Yb + SB * rr + 64 * q;
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int k = 0; k < 64; k += 2) {
                    a0 += l[k] * yb[k];
                    a1 += l[k + 1] * yb[k + 1];
                }
                part[(q * 16 + rr) * 64 + lane] = a0 + a1;
            }
        }
        __syncthreads();
        if (q == 0 && i < f)
            for (int rr = 0; rr < nr; ++rr) {
                if (active && !active[rg + rr]) continue;
                double acc = 0.0 + part[rr * 64 + lane];  // as a sum started at zero
                for (int w = 1; 64 * w < nbJ; ++w) acc += part[(w * 16 + rr) * 64 + lane];
                Ys[i + (int64_t)(rg + rr) * S.ytot] -= acc;
            }
    }
}

__global__ __launch_bounds__(256) void k_sffin(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                               const int32_t* active) {
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, i = 256 * t.k0 + threadIdx.x;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s];
    if (i >= f) return;
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        const double* y = S.Y + D.yoff[s] + (int64_t)r * S.ytot;
        if (i >= p) {
            S.ub[D.ub_off[s] + (i - p) + (int64_t)r * D.ub_total] = y[i];
            continue;
        }
        const int ty = D.ptype[c0 + i];
        double v;
        if (ty == 0) v = y[i] / D.dval[c0 + i];
        else if (ty == 1) {
            const double a = D.dval[c0 + i], b = D.doff[c0 + i], c = D.dval[c0 + i + 1];
            v = (c * y[i] - b * y[i + 1]) / (a * c - b * b);
        } else {
            const double a = D.dval[c0 + i - 1], b = D.doff[c0 + i - 1], c = D.dval[c0 + i];
            v = (a * y[i] - b * y[i - 1]) / (a * c - b * b);
        }
        S.xw[(int64_t)r * D.N + c0 + D.lperm[c0 + i]] = v;
    }
}

__global__ __launch_bounds__(256) void k_sbload(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                                const int32_t* active) {
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, i = 256 * t.k0 + threadIdx.x;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s];
    if (i >= f) return;
    const int32_t src = i < p ? c0 + D.lperm[c0 + i] : D.rows[D.sn_rowptr[s] + i];
    for (int r = 0; r < S.nrhs; ++r)
        if (!active || active[r]) S.Y[D.yoff[s] + i + (int64_t)r * S.ytot] = S.xw[(int64_t)r * D.N + src];
}

// partial sums over one 256-row chunk below block J: P[(b * SB + k) * nrhs + r] =
// sum_i L(i, k0 + k) y_i[r] for 64 of the block's columns (sub-block blockIdx.y); the rows
// are taken in 64-row tiles loaded coalesced (lane = row) and summed through LDS (lane =
// column), right-hand sides eight at a time
__global__ __launch_bounds__(256) void k_sbpart(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                                const int32_t* active) {
    __shared__ double Lt[64 * 65];
    __shared__ double Yt[8 * 64];
    __shared__ double red[4 * 64 * 8];
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, kJ = SB * t.k0;
    const int f = D.sn_f[s], p = D.sn_p[s], ld = D.sn_ld[s];
    const int k1 = min(kJ + SB, p), nbJ = k1 - kJ;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const double* F = D.front + D.sn_off[s];
    const double* Ys = S.Y + D.yoff[s];
    const int r0 = k1 + 256 * t.a, r1 = min(f, r0 + 256);
    {
        const int a = (int)blockIdx.y;  // the block's 64-column sub-block
        if (64 * a >= nbJ) return;
        const int k0 = kJ + 64 * a, nb = min(64, nbJ - 64 * a);
        for (int rg = 0; rg < S.nrhs; rg += 8) {
            const int nr = min(8, S.nrhs - rg);
            double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int i0 = r0; i0 < r1; i0 += 64) {
                double v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int k = wv + 4 * q, i = i0 + lane;
                    v[q] = (k < nb && i < r1) ? F[i + (int64_t)(k0 + k) * ld] : 0.0;
                }
                __syncthreads();  // the previous tile's sums are done with Lt, Yt
#pragma unroll
                for (int q = 0; q < 16; ++q) Lt[(wv + 4 * q) * 65 + lane] = v[q];
                for (int idx = tid; idx < 8 * 64; idx += 256) {
                    const int i = idx & 63, rr = idx >> 6;
                    Yt[idx] = (rr < nr && i0 + i < r1) ? Ys[i0 + i + (int64_t)(rg + rr) * S.ytot] : 0.0;
                }
                __syncthreads();
                for (int q = 0; q < 16; ++q) {  // rows wv + 4q of the tile, column lane
                    const int i = wv + 4 * q;
                    const double lv = Lt[lane * 65 + i];
#pragma unroll
                    for (int rr = 0; rr < 8; ++rr) acc[rr] += lv * Yt[rr * 64 + i];
                }
            }
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) red[(wv * 64 + lane) * 8 + rr] = acc[rr];
            __syncthreads();
            if (wv == 0)
                for (int rr = 0; rr < nr; ++rr) {
                    const double sum = ((red[(0 * 64 + lane) * 8 + rr] + red[(1 * 64 + lane) * 8 + rr]) +
                                        red[(2 * 64 + lane) * 8 + rr]) + red[(3 * 64 + lane) * 8 + rr];
                    S.P[((int64_t)t.b * SB + 64 * a + lane) * S.nrhs + rg + rr] = sum;
                }
            __syncthreads();
        }
    }
}

// backward: y_J <- L_JJ^{-T} (y_J - sum of the block's partial sums, chunks in fixed order),
// sub-blocks of 64 from the last: y_a -= L_ba^T y_b for the later sub-blocks b of the block
// (L_ba staged through LDS, four row quarters summed in a fixed order), then the sub-block's
// own triangular solve; right-hand sides eight at a time
__global__ __launch_bounds__(256) void k_sbdiag(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                                const int32_t* active) {
    __shared__ double Lb[64 * 65];
    __shared__ double yb[SB * 8];
    __shared__ double part[4 * 64 * 8];
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, kJ = SB * t.k0;
    const int p = D.sn_p[s], ld = D.sn_ld[s];
    const int nbJ = min(SB, p - kJ);
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const double* F = D.front + D.sn_off[s];
    double* Ys = S.Y + D.yoff[s] + kJ;
    const int nsub = (nbJ + 63) / 64;
    for (int rg = 0; rg < S.nrhs; rg += 8) {
        const int nr = min(8, S.nrhs - rg);
        for (int idx = tid; idx < SB * 8; idx += 256) {
            const int i = idx & (SB - 1), rr = idx / SB;
            double v = 0.0;
            if (i < nbJ && rr < nr) {
                double sum = 0.0;
                for (int c = 0; c < t.b; ++c) sum += S.P[((int64_t)(t.a + c) * SB + i) * S.nrhs + rg + rr];
                v = Ys[i + (int64_t)(rg + rr) * S.ytot] - sum;
            }
            yb[idx] = v;
        }
        for (int a = nsub - 1; a >= 0; --a) {
            const int nb = min(64, nbJ - 64 * a);
            for (int b = a + 1; b < nsub; ++b) {  // y_a -= L_ba^T y_b
                const int nbb = min(64, nbJ - 64 * b);
                double v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {  // L(64 b + lane, 64 a + k), k = wv + 4 q
                    const int k = wv + 4 * q;
                    v[q] = (k < nb && lane < nbb) ? F[kJ + 64 * b + lane + (int64_t)(kJ + 64 * a + k) * ld] : 0.0;
                }
                __syncthreads();  // earlier readers of Lb, part and yb are done
#pragma unroll
                for (int q = 0; q < 16; ++q) Lb[(wv + 4 * q) * 65 + lane] = v[q];
                __syncthreads();
                // thread (k = lane, quarter wv): rows 16 wv .. 16 wv + 15 of L_ba column k
                for (int rr = 0; rr < nr; ++rr) {
                    const double* yv = yb + SB * rr + 64 * b;
                    double acc = 0.0;
#pragma unroll
                    for (int u = 0; u < 16; ++u) acc += Lb[lane * 65 + 16 * wv + u] * yv[16 * wv + u];
                    part[(wv * 64 + lane) * 8 + rr] = acc;
                }
                __syncthreads();
                if (wv == 0 && lane < nb)
                    for (int rr = 0; rr < nr; ++rr)
                        yb[SB * rr + 64 * a + lane] -= ((part[(0 * 64 + lane) * 8 + rr] + part[(1 * 64 + lane) * 8 + rr]) +
                                                         part[(2 * 64 + lane) * 8 + rr]) + part[(3 * 64 + lane) * 8 + rr];
            }
            __syncthreads();
            {
                BlockRegs<64> bl;
                load_inv<64>(bl, D.linv + D.inv_off[s] + 4096 * (int64_t)(4 * t.k0 + a), nb, tid);
                store_block<64>(Lb, bl, tid);
            }
            __syncthreads();
            for (int rr = 0; rr < nr; ++rr) {  // rr and active[] are the same for the workgroup
                if (active && !active[rg + rr]) continue;
                block_inv_apply<64, true>(Lb, yb + SB * rr + 64 * a, nb, part, tid);
            }
        }
        __syncthreads();
        for (int idx = tid; idx < SB * 8; idx += 256) {
            const int i = idx & (SB - 1), rr = idx / SB;
            if (i < nbJ && rr < nr && (!active || active[rg + rr])) Ys[i + (int64_t)(rg + rr) * S.ytot] = yb[idx];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_sbstore(DevPlan D, DevSolve S, const Task* tasks, int64_t t0,
                                                 const int32_t* active) {
    if (big_inactive(S, active)) return;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, i = 256 * t.k0 + threadIdx.x;
    const int p = D.sn_p[s], c0 = D.sn_ptr[s];
    if (i >= p) return;
    for (int r = 0; r < S.nrhs; ++r)
        if (!active || active[r]) S.xw[(int64_t)r * D.N + c0 + D.lperm[c0 + i]] = S.Y[D.yoff[s] + i + (int64_t)r * S.ytot];
}

// One level of the supernodal tree per launch: the kernel boundary orders the levels.
// NBM: a bound on the pivot count of every supernode of the level, capped at 64 (sizes the
// register blocks, so levels of small supernodes keep many workgroups per CU).
template <int NBM>
__global__ __launch_bounds__(256) void k_fwd(DevPlan D, DevSolve S, const int32_t* lvl_sn, int64_t base,
                                             const int32_t* active) {
    extern __shared__ double dyn[];
    __shared__ double Lb[NBM * (NBM + 1)];
    __shared__ double part[256];
    fwd_supernode<NBM>(D, S, lvl_sn[base + blockIdx.x], active, dyn, Lb, part);
}

template <int NBM>
__global__ __launch_bounds__(256) void k_bwd(DevPlan D, DevSolve S, const int32_t* lvl_sn, int64_t base,
                                             const int32_t* active) {
    extern __shared__ double dyn[];
    __shared__ double Lb[NBM * (NBM + 1)];
    __shared__ double part[4 * 64];
    __shared__ double Lt[NBM * 65];
    bwd_supernode<NBM>(D, S, lvl_sn[base + blockIdx.x], active, dyn, Lb, part, Lt);
}

// Inverse of one unit lower diagonal block (64 pivots) of L, for the one-workgroup solves:
// one wavefront, lane c computes column c of the inverse by forward substitution with the
// block in LDS (every lane reads the same entry: broadcast), four partial sums per row.
__global__ __launch_bounds__(64) void k_inv(DevPlan D, const Task* tasks) {
    __shared__ double Ls[64 * 65];  // Ls[k * 65 + j] = L(k, j), strictly lower, zero elsewhere
    const Task t = tasks[blockIdx.x];
    const int s = t.s, k0 = 64 * t.k0, lane = threadIdx.x;
    if (gated_off(D, s)) return;
    const int p = D.sn_p[s], ld = D.sn_ld[s];
    const int nb = min(64, p - k0);
    const double* F = D.front + D.sn_off[s] + k0 + (int64_t)k0 * ld;
    for (int j0 = 0; j0 < 64; j0 += 8) {  // column j of the block, lane = row; eight in flight
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = j0 + u;
            v[u] = (lane < nb && j < nb && lane > j) ? F[lane + (int64_t)j * ld] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) Ls[lane * 65 + j0 + u] = v[u];
    }
    __syncthreads();
    const int c = lane;
    double x[64];
#pragma unroll
    for (int k = 0; k < 64; ++k) {
        double a0 = k == c ? 1.0 : 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (k < nb) {
#pragma unroll
            for (int j = 0; j + 3 < k; j += 4) {
                a0 -= Ls[k * 65 + j] * x[j];
                a1 -= Ls[k * 65 + j + 1] * x[j + 1];
                a2 -= Ls[k * 65 + j + 2] * x[j + 2];
                a3 -= Ls[k * 65 + j + 3] * x[j + 3];
            }
#pragma unroll
            for (int j = k & ~3; j < k; ++j) a0 -= Ls[k * 65 + j] * x[j];
        }
        x[k] = (a0 + a1) + (a2 + a3);
    }
    double* out = D.linv + D.inv_off[s] + 4096 * (int64_t)t.k0;
    if (c < nb) {
#pragma unroll
        for (int k = 0; k < 64; ++k)
            if (k < nb) out[k + (int64_t)c * nb] = k >= c ? x[k] : 0.0;
    }
}

// Levels whose fronts all have f <= 64: one wavefront per supernode, four per workgroup.
// Lane i holds y_i (pivot rows in post-pivot order).  Forward: lane i gathers pre-pivot row
// lperm(i) directly, so no permutation step is needed; each pivot k broadcasts y_k by readlane.
template <int PM>
__global__ __launch_bounds__(256) void k_fwd_wave(DevPlan D, DevSolve S, const int32_t* lvl_sn, int64_t base,
                                                  int count, const int32_t* active) {
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (w >= count) return;
    const int s = __builtin_amdgcn_readfirstlane(lvl_sn[base + w]);
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const double* F = D.front + D.sn_off[s];
    const bool on = lane < f;
    const int t = lane < p ? D.lperm[c0 + lane] : lane;  // pre-pivot row at position lane
    double l[PM];
#pragma unroll
    for (int k = 0; k < PM; ++k) l[k] = (k < p && on && lane > k) ? F[lane + (int64_t)k * ld] : 0.0;
    int ty = 0;
    double da = 1.0, db = 0.0, dc = 1.0;
    if (lane < p) {
        ty = D.ptype[c0 + lane];
        const int k2 = ty == 2 ? lane - 1 : lane;
        da = D.dval[c0 + k2];
        db = ty ? D.doff[c0 + k2] : 0.0;
        dc = ty ? D.dval[c0 + k2 + 1] : 1.0;
    }
    const int64_t* gp = D.fg_ptr + D.sn_rowptr[s];
    const int64_t q0 = on ? gp[t] : 0, q1 = on ? gp[t + 1] : 0;
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        double* xw = S.xw + (int64_t)r * D.N;
        double* ub = S.ub + (int64_t)r * D.ub_total;
        double y = (on && lane < p) ? xw[c0 + t] : 0.0;
        for (int64_t q = q0; q < q1; q += 4) {  // four contributions in flight, added in list order
            int64_t src[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) src[j] = q + j < q1 ? D.fg_src[q + j] : -1;
            double val[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) val[j] = src[j] >= 0 ? ub[src[j]] : 0.0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (src[j] >= 0) y += val[j];
        }
#pragma unroll
        for (int k = 0; k < PM; ++k) {  // every pivot, the last one too: rows below are lanes >= p
            if (k < p) {
                const double yk = readlane_d(y, k);
                if (lane > k) y -= l[k] * yk;
            }
        }
        const double yn = shfl_d(y, min(lane + 1, 63)), yp = shfl_d(y, max(lane - 1, 0));
        if (on && lane >= p) ub[D.ub_off[s] + lane - p] = y;
        if (lane < p) {
            double x;
            if (ty == 0) x = y / da;
            else if (ty == 1) x = (dc * y - db * yn) / (da * dc - db * db);
            else x = (da * y - db * yp) / (da * dc - db * db);
            xw[c0 + t] = x;
        }
    }
}

// Backward solve, one wavefront per supernode: lane j < p accumulates sum_i L(i, j) y_i,
// first over the rows below the pivot block (its own column of L, eight rows per trip),
// then over the pivot block from the last pivot up, one readlane per pivot.
template <int PM>
__global__ __launch_bounds__(256) void k_bwd_wave(DevPlan D, DevSolve S, const int32_t* lvl_sn, int64_t base,
                                                  int count, const int32_t* active) {
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    if (w >= count) return;
    const int s = __builtin_amdgcn_readfirstlane(lvl_sn[base + w]);
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const double* F = D.front + D.sn_off[s];
    const double* Fj = F + (int64_t)min(lane, p - 1) * ld;  // column lane of L (lanes < p)
    const bool on = lane < f;
    const int src = lane < p ? c0 + D.lperm[c0 + lane] : (on ? D.rows[D.sn_rowptr[s] + lane] : 0);
    double c[PM];  // c[k] = L(k, lane): row k of the pivot block, column lane
#pragma unroll
    for (int k = 0; k < PM; ++k) c[k] = (k < p && lane < k) ? Fj[k] : 0.0;
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        double* xw = S.xw + (int64_t)r * D.N;
        double y = on ? xw[src] : 0.0;
        double a0 = 0.0, a1 = 0.0;
        for (int i0 = p; i0 < f; i0 += 8) {
            double lv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) lv[u] = (lane < p && i0 + u < f) ? Fj[i0 + u] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; u += 2) {
                if (i0 + u < f) a0 += lv[u] * readlane_d(y, i0 + u);
                if (i0 + u + 1 < f) a1 += lv[u + 1] * readlane_d(y, i0 + u + 1);
            }
        }
        double acc = a0 + a1;
#pragma unroll
        for (int k = PM - 1; k >= 0; --k) {
            if (k >= p) continue;
            if (lane == k) y -= acc;
            const double yk = readlane_d(y, k);
            acc += c[k] * yk;  // c[k] = 0 for lanes >= k
        }
        if (lane < p) xw[src] = y;
    }
}

// r = b - K_static x and (|K||x|)_i in original numbering, from A, Theta, rho, delta
// (AS) or from the K values (NE); per-block maxima of |r|, |x|, |b|.
// AS: the sums over the long columns of A (more than LONG_COL entries, e.g. dense columns)
// that the residual and the Krylov products need for the primal rows, one workgroup per (long
// column, right-hand side): sum_i A_ij x_{n+i} and sum_i |A_ij||x_{n+i}|, each thread over a
// fixed stride of the column, then a fixed-order tree (bitwise reproducible).  One thread per
// primal row would take the whole column serially.
__global__ __launch_bounds__(256) void k_long_cols(DevPlan D, const double* xin, double* lsum,
                                                   const int32_t* act) {
    __shared__ double red[2][256];
    const int q = blockIdx.x, r = blockIdx.y;
    if (act && !act[r]) return;
    const int j = D.long_col[q];
    const double* x = xin + (int64_t)r * D.N + D.n;
    double s = 0.0, sa = 0.0;
    for (int64_t e = D.acp[j] + threadIdx.x; e < D.acp[j + 1]; e += 256) {
        const double a = D.aval[e], v = x[D.ari[e]];
        s += a * v;
        sa += fabs(a) * fabs(v);
    }
    red[0][threadIdx.x] = s;
    red[1][threadIdx.x] = sa;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 2) lsum[2 * ((int64_t)r * D.nlong + q) + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_residual(DevPlan D, DevSolve S, const double* xin) {
    __shared__ double red[3][256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    const double* x = xin + (int64_t)r * D.N;
    const double* b = S.b + (int64_t)r * D.N;
    double ar = 0.0, ax = 0.0, ab = 0.0;
    if (i < D.N) {
        const int sys = D.sys_old[i];
        const double rho = D.rho_sys[sys], delta = D.delta_sys[sys];
        double kx = 0.0, akx = 0.0;
        if (D.mode == 1) {
            if (i < D.n) {
                const double dj = D.has_q ? -((D.dinv[i] + q_diag(D, i)) + rho) : -(D.dinv[i] + rho);
                kx = dj * x[i];
                akx = fabs(dj) * fabs(x[i]);
                if (D.has_q)
                    for (int64_t e = D.qfcp[i]; e < D.qfcp[i + 1]; ++e) {
                        const int k = D.qfri[e];
                        if (k == i) continue;
                        const double q = -D.qval[D.qfsrc[e]];
                        kx += q * x[k];
                        akx += fabs(q) * fabs(x[k]);
                    }
                // four entries per trip, their loads in flight together, added in order; a long
                // column's sums come from k_long_cols
                const int lq = D.nlong ? D.long_of[i] : -1;
                if (lq >= 0) {
                    kx += S.lsum[2 * ((int64_t)r * D.nlong + lq)];
                    akx += S.lsum[2 * ((int64_t)r * D.nlong + lq) + 1];
                }
                const int64_t e1 = lq >= 0 ? D.acp[i] : D.acp[i + 1];
                for (int64_t e = D.acp[i]; e < e1; e += 4) {
                    double a[4], xv[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const bool on = e + j < e1;
                        a[j] = on ? D.aval[e + j] : 0.0;
                        xv[j] = on ? x[D.n + D.ari[e + j]] : 0.0;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (e + j < e1) {
                            kx += a[j] * xv[j];
                            akx += fabs(a[j]) * fabs(xv[j]);
                        }
                }
            } else {
                const int row = i - D.n;
                const int64_t q1 = D.arp[row + 1];
                for (int64_t q = D.arp[row]; q < q1; q += 4) {
                    int32_t ej[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) ej[j] = q + j < q1 ? D.are[q + j] : -1;
                    double a[4], xv[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        a[j] = ej[j] >= 0 ? D.aval[ej[j]] : 0.0;
                        xv[j] = ej[j] >= 0 ? x[D.acol[ej[j]]] : 0.0;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (ej[j] >= 0) {
                            kx += a[j] * xv[j];
                            akx += fabs(a[j]) * fabs(xv[j]);
                        }
                }
                kx += delta * x[i];
                akx += delta * fabs(x[i]);
            }
        } else {
            // four entries of row i per trip: their indices, then their values, in flight
            // together; added in list order
            const int64_t q1 = D.krs_ptr[i + 1];
            for (int64_t q = D.krs_ptr[i]; q < q1; q += 4) {
                int o[4];
                int32_t ent[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const bool on = q + j < q1;
                    o[j] = on ? D.krs_other[q + j] : -1;
                    ent[j] = on ? D.krs_ent[q + j] : -1;
                }
                double v[4], xv[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v[j] = o[j] >= 0 ? D.kval[ent[j]] : 0.0;
                    xv[j] = o[j] >= 0 ? x[o[j]] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (o[j] >= 0) {
                        const double vj = o[j] == i ? v[j] + delta : v[j];
                        kx += vj * xv[j];
                        akx += fabs(vj) * fabs(xv[j]);
                    }
            }
        }
        const double rv = b[i] - kx;
        S.r[i + (int64_t)r * D.N] = rv;
        S.d[i + (int64_t)r * D.N] = akx;
        ar = fabs(rv);
        ax = fabs(x[i]);
        ab = fabs(b[i]);
    }
    red[0][threadIdx.x] = ar;
    red[1][threadIdx.x] = ax;
    red[2][threadIdx.x] = ab;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = nmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 3) S.part[(int64_t)r * 3 * S.nblk + threadIdx.x * S.nblk + blockIdx.x] = red[threadIdx.x][0];
}

// The refinement decision of unit u (system, rhs) from its new backward errors: record them,
// count the step, and keep refining while the target is not met, the error still halves and
// steps remain; a step that does not improve is undone (returns 1: restore the previous x).
__device__ inline int berr_decide(DevSolve& S, int u, int phase, double nw, double cw, double target,
                                  int max_steps) {
    double* be = S.berr + 4 * u;
    if (phase == 0) {
        be[0] = nw;
        be[1] = cw;
        be[2] = nw;
        S.steps[u] = 0;
        S.active[u] = (nw > target && max_steps > 0) ? 1 : 0;
        return 0;
    }
    const double prev = be[0];
    S.steps[u] += 1;
    if (!(nw < prev)) {  // no improvement: keep the previous iterate
        S.active[u] = 0;
        return 1;
    }
    const bool stagnating = nw > 0.5 * prev;
    be[0] = nw;
    be[1] = cw;
    S.active[u] = (!stagnating && nw > target && S.steps[u] < max_steps) ? 1 : 0;
    return 0;
}

// Backward errors (normwise in the infinity norm; componentwise with the small-denominator
// substitution of Arioli, Demmel and Duff) and the refinement decision for each rhs.
// phase 0: after the first solve; phase 1: after a refinement step.
__global__ __launch_bounds__(1024) void k_berr(DevPlan D, DevSolve S, int phase, double target, int max_steps) {
    __shared__ double red[4][1024];
    const int q = blockIdx.x, r = blockIdx.y, u = r * D.nsys + q;  // system q, rhs r
    if (phase == 1 && !S.active[u]) return;
    const int64_t* rg = D.sys_rng + 4 * q;
    const double* rr = S.r + (int64_t)r * D.N;
    const double* akx = S.d + (int64_t)r * D.N;
    const double* b = S.b + (int64_t)r * D.N;
    const double* x = S.x + (int64_t)r * D.N;
    double mr = 0.0, mx = 0.0, mb = 0.0;
    for (int part = 0; part < 2; ++part)
#pragma unroll 8
        for (int64_t i = rg[2 * part] + threadIdx.x; i < rg[2 * part + 1]; i += 1024) {
            mr = nmax(mr, fabs(rr[i]));
            mx = nmax(mx, fabs(x[i]));
            mb = nmax(mb, fabs(b[i]));
        }
    red[0][threadIdx.x] = mr;
    red[1][threadIdx.x] = mx;
    red[2][threadIdx.x] = mb;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int v = 0; v < 3; ++v) red[v][threadIdx.x] = nmax(red[v][threadIdx.x], red[v][threadIdx.x + w]);
        __syncthreads();
    }
    const double rmax = red[0][0], xmax = red[1][0], bmax = red[2][0];
    const double u64 = 1.1102230246251565e-16;
    double cm = 0.0;
    for (int part = 0; part < 2; ++part)
#pragma unroll 8
        for (int64_t i = rg[2 * part] + threadIdx.x; i < rg[2 * part + 1]; i += 1024) {
            double den = akx[i] + fabs(b[i]);
            if (den <= 1000.0 * D.N * u64 * (D.rowsum[i] * xmax + fabs(b[i]))) den = akx[i] + xmax * D.rowsum[i];
            const double c = den > 0 ? fabs(rr[i]) / den : (rr[i] == 0 ? 0.0 : INFINITY);
            cm = nmax(cm, c);
        }
    __syncthreads();
    red[3][threadIdx.x] = cm;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[3][threadIdx.x] = nmax(red[3][threadIdx.x], red[3][threadIdx.x + w]);
        __syncthreads();
    }
    const double cw = red[3][0];
    const double den = D.knorm_sys[q] * xmax + bmax;
    const double nw = den > 0 ? rmax / den : (rmax == 0 ? 0.0 : INFINITY);
    __shared__ int restore;
    if (threadIdx.x == 0) restore = berr_decide(S, u, phase, nw, cw, target, max_steps);
    __syncthreads();
    if (restore) {
        double* xw = S.x + (int64_t)r * D.N;
        const double* xb = S.xbak + (int64_t)r * D.N;
        for (int part = 0; part < 2; ++part)
            for (int64_t i = rg[2 * part] + threadIdx.x; i < rg[2 * part + 1]; i += 1024) xw[i] = xb[i];
    }
}

// One system (nsys == 1) over many workgroups: the maxima of |r|, |x| and |b| come from the
// residual kernel's per-block partials; each workgroup takes the componentwise ratio over its
// 256 rows (section 3 of the partials), and one workgroup per rhs combines and decides.
__device__ inline double block_max256(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = nmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double m = red[0];
    __syncthreads();
    return m;
}

__global__ __launch_bounds__(256) void k_berr_cw(DevPlan D, DevSolve S, int phase) {
    __shared__ double red[256];
    const int r = blockIdx.y;
    if (phase == 1 && !S.active[r]) return;
    const double* px = S.part + (int64_t)r * 3 * S.nblk + S.nblk;  // per-block max |x|
    double m = 0.0;
    for (int j = threadIdx.x; j < S.nblk; j += 256) m = nmax(m, px[j]);
    const double xmax = block_max256(m, red);
    const double u64 = 1.1102230246251565e-16;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double c = 0.0;
    if (i < D.N) {
        const double rr = S.r[i + (int64_t)r * D.N], bi = fabs(S.b[i + (int64_t)r * D.N]);
        const double akx = S.d[i + (int64_t)r * D.N];
        double den = akx + bi;
        if (den <= 1000.0 * D.N * u64 * (D.rowsum[i] * xmax + bi)) den = akx + xmax * D.rowsum[i];
        c = den > 0 ? fabs(rr) / den : (rr == 0 ? 0.0 : INFINITY);
    }
    const double cm = block_max256(c, red);
    if (threadIdx.x == 0) S.part[(int64_t)3 * S.nblk * S.nrhs + (int64_t)r * S.nblk + blockIdx.x] = cm;
}

__global__ __launch_bounds__(256) void k_berr_fin(DevPlan D, DevSolve S, int phase, double target, int max_steps) {
    __shared__ double red[256];
    __shared__ int restore;
    const int r = blockIdx.x;
    if (phase == 1 && !S.active[r]) return;
    const double* pr = S.part + (int64_t)r * 3 * S.nblk;
    const double* pc = S.part + (int64_t)3 * S.nblk * S.nrhs + (int64_t)r * S.nblk;
    double mr = 0.0, mx = 0.0, mb = 0.0, mc = 0.0;
    for (int j = threadIdx.x; j < S.nblk; j += 256) {
        mr = nmax(mr, pr[j]);
        mx = nmax(mx, pr[S.nblk + j]);
        mb = nmax(mb, pr[2 * S.nblk + j]);
        mc = nmax(mc, pc[j]);
    }
    const double rmax = block_max256(mr, red), xmax = block_max256(mx, red);
    const double bmax = block_max256(mb, red), cw = block_max256(mc, red);
    const double den = D.knorm_sys[0] * xmax + bmax;
    const double nw = den > 0 ? rmax / den : (rmax == 0 ? 0.0 : INFINITY);
    if (threadIdx.x == 0) restore = berr_decide(S, r, phase, nw, cw, target, max_steps);
    __syncthreads();
    if (restore) {
        double* xw = S.x + (int64_t)r * D.N;
        const double* xb = S.xbak + (int64_t)r * D.N;
        for (int64_t i = threadIdx.x; i < D.N; i += 256) xw[i] = xb[i];
    }
}

// ---------------------------------------------------------------- Krylov refinement
// Vectors are N x nrhs blocks in original numbering; a basis V holds blocks j = 0, 1, ...
// at V + j * N * nrhs.  Reductions run in a fixed order (one workgroup per output).

// out = K_static v, from A, Theta, rho, delta (AS) or from the K values (NE).
__global__ __launch_bounds__(256) void k_matvec(DevPlan D, const double* vin, double* out, int nrhs,
                                                const double* lsum, const int32_t* act) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N || r >= nrhs || (act && !act[r])) return;
    const double* v = vin + (int64_t)r * D.N;
    const int sys = D.sys_old[i];
    const double rho = D.rho_sys[sys], delta = D.delta_sys[sys];
    double kx = 0.0;
    if (D.mode == 1) {
        if (i < D.n) {
            kx = (D.has_q ? -((D.dinv[i] + q_diag(D, i)) + rho) : -(D.dinv[i] + rho)) * v[i];
            if (D.has_q)
                for (int64_t e = D.qfcp[i]; e < D.qfcp[i + 1]; ++e)
                    if (D.qfri[e] != i) kx -= D.qval[D.qfsrc[e]] * v[D.qfri[e]];
            const int lq = D.nlong ? D.long_of[i] : -1;
            if (lq >= 0) kx += lsum[2 * ((int64_t)r * D.nlong + lq)];
            else
                for (int64_t e = D.acp[i]; e < D.acp[i + 1]; ++e) kx += D.aval[e] * v[D.n + D.ari[e]];
        } else {
            const int row = i - D.n;
            for (int64_t q = D.arp[row]; q < D.arp[row + 1]; ++q) {
                const int32_t e = D.are[q];
                kx += D.aval[e] * v[D.acol[e]];
            }
            kx += delta * v[i];
        }
    } else {
        for (int64_t q = D.krs_ptr[i]; q < D.krs_ptr[i + 1]; ++q) {
            const int o = D.krs_other[q];
            double kv = D.kval[D.krs_ent[q]];
            if (o == i) kv += delta;
            kx += kv * v[o];
        }
    }
    out[i + (int64_t)r * D.N] = kx;
}

// out[j * nrhs + r] = <V_j(:, r), w(:, r)> for j < nv.
// Krylov vectors are N x nrhs blocks (original numbering); the refinement unit u = r * nsys + q
// is right-hand side r of system q, whose entries are the index ranges [a0, a1) and [b0, b1)
// of sys_rng.  Per unit, dots: out[j * U + u] = V_j(:, r) . w(:, r) over the unit's entries
// (U = nrhs * nsys), fixed-order tree; units with act[u] == 0 are skipped (act may be NULL).
__global__ __launch_bounds__(256) void k_dots(DevPlan D, const double* V, int nv, const double* w, double* out,
                                              int nrhs, const int32_t* act) {
    __shared__ double red[256];
    const int j = blockIdx.x, u = blockIdx.y;
    if (act && !act[u]) return;
    const int r = u / D.nsys, q = u % D.nsys;
    const int64_t N = D.N;
    const double* a = V + ((int64_t)j * nrhs + r) * N;
    const double* b = w + (int64_t)r * N;
    double acc = 0.0;
    for (int h = 0; h < 2; ++h) {
        const int64_t i0 = D.sys_rng[4 * q + 2 * h], i1 = D.sys_rng[4 * q + 2 * h + 1];
        for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc += a[i] * b[i];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)j * nrhs * D.nsys + u] = red[0];
}

// w(:, r) -= sum_{j < nv} h[j * U + u] V_j(:, r)   (sign = 1), or
// w(:, r)  = sum_{j < nv} h[j * U + u] V_j(:, r)   (sign = 0), entry i taking the unit u of its
// own system; units with act[u] == 0 are left alone (act may be NULL), and nvr (may be NULL)
// caps nv per unit.
__global__ void k_vcombine(DevPlan D, const double* V, int nv, const double* h, double* w, int nrhs, int sign,
                           const int32_t* act, const int32_t* nvr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N) return;
    const int u = r * D.nsys + D.sys_old[i];
    if (act && !act[u]) return;
    const int64_t U = (int64_t)nrhs * D.nsys;
    const int nj = nvr ? min(nv, nvr[u]) : nv;
    double acc = 0.0;
    for (int j = 0; j < nj; ++j) acc += h[j * U + u] * V[((int64_t)j * nrhs + r) * D.N + i];
    double* wi = w + (int64_t)r * D.N + i;
    *wi = sign ? *wi - acc : acc;
}

// dst(:, r) = src(:, r) / sqrt(nrm2[u]) per unit (0 where the norm is 0 or not finite).
__global__ void k_vscale(DevPlan D, const double* src, const double* nrm2, double* dst, int nrhs,
                         const int32_t* act) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N) return;
    const int u = r * D.nsys + D.sys_old[i];
    if (act && !act[u]) return;
    const double nn = sqrt(nrm2[u]);
    dst[(int64_t)r * D.N + i] = (nn > 0.0 && nn < INFINITY) ? src[(int64_t)r * D.N + i] / nn : 0.0;
}

// Per rhs: whether any system still refines (the solve kernels' gate in a batch).
__global__ void k_any_active(DevPlan D, DevSolve S) {
    const int r = blockIdx.x;
    int any = 0;
    for (int q = threadIdx.x; q < D.nsys; q += blockDim.x) any |= S.active[r * D.nsys + q];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) S.ract[r] = any;
}

__global__ void k_refine_begin(DevPlan D, DevSolve S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N || !S.active[r * D.nsys + D.sys_old[i]]) return;
    S.xbak[i + (int64_t)r * D.N] = S.x[i + (int64_t)r * D.N];
}

__global__ void k_refine_update(DevPlan D, DevSolve S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N || !S.active[r * D.nsys + D.sys_old[i]]) return;
    S.x[i + (int64_t)r * D.N] += S.d[i + (int64_t)r * D.N];
}

// AS: split x into (dx, dy).  NE: dy = x, dx = theta~ (A^T dy - r7) (Section 3).
__global__ void k_recover(DevPlan D, DevSolve S, const double* r7, double* dx, double* dy) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    const double* x = S.x + (int64_t)r * D.N;
    if (D.mode == 1) {
        if (t < D.n) dx[t + (int64_t)r * D.n] = x[t];
        if (t < D.m) dy[t + (int64_t)r * D.m] = x[D.n + t];
    } else {
        if (t < D.m) dy[t + (int64_t)r * D.m] = x[t];
        if (t < D.n) {
            double s = 0.0;
            for (int64_t e = D.acp[t]; e < D.acp[t + 1]; ++e) s += D.aval[e] * x[D.ari[e]];
            dx[t + (int64_t)r * D.n] = D.dinv[t] * (s - (r7 ? r7[t + (int64_t)r * D.n] : 0.0));
        }
    }
}

// GMRES on K_static M (right preconditioning by the factor, M = (L D L^T)^{-1}) for the
// correction of one refinement step, one Krylov process per refinement unit u (right-hand
// side x system: the systems of a batch are independent, so each gets its own coefficients),
// the Hessenberg matrix reduced by Givens rotations as the Arnoldi process goes, all on the
// device with one thread per unit.  State per unit (strides GM_M + 1 or GM_M): beta =
// ||r_u||_2, the rotated right-hand side g, the rotations (c, s), the triangular factor R
// (GM_M x GM_M, column j written at step j), the number of Krylov vectors taken kr, and act = 1
// while the unit takes more steps; ract per rhs: some unit of it does.
__global__ void k_gm_start(DevGmres G, const int32_t* gate, int nu) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu) return;
    const double beta = sqrt(G.nrm[u]);
    const int on = gate[u] && beta > 0.0 && beta < INFINITY;
    G.act[u] = on;
    G.kr[u] = 0;
    G.beta[u] = beta;
    for (int i = 0; i <= GM_M; ++i) G.g[u * (GM_M + 1) + i] = i == 0 ? beta : 0.0;
}

// Step j: the new Hessenberg column h (both Gram-Schmidt passes' coefficients summed, and
// ||w||_2 below), the earlier rotations applied to it, a new rotation that zeroes h[j + 1],
// and the estimate |g[j + 1]| of the residual norm; the unit stops at tol * beta, at a
// breakdown (h[j + 1] = 0: the Krylov space holds the solution) or on a non-finite value.
__global__ void k_gm_rotate(DevGmres G, int j, int nu, double tol) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu || !G.act[u]) return;
    double col[GM_M + 1];
    for (int i = 0; i <= j; ++i) col[i] = G.h1[(int64_t)i * nu + u] + G.h2[(int64_t)i * nu + u];
    col[j + 1] = sqrt(G.nrm[u]);
    double* cs = G.cs + (int64_t)u * GM_M;
    double* sn = G.sn + (int64_t)u * GM_M;
    for (int i = 0; i < j; ++i) {
        const double a = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = a;
    }
    const double a = col[j], b = col[j + 1];
    const double den = hypot(a, b);
    const double c = den > 0.0 ? a / den : 1.0, sg = den > 0.0 ? b / den : 0.0;
    cs[j] = c;
    sn[j] = sg;
    col[j] = den;
    for (int i = 0; i <= j; ++i) G.R[((int64_t)u * GM_M + j) * GM_M + i] = col[i];
    double* g = G.g + (int64_t)u * (GM_M + 1);
    const double gj = g[j];
    g[j] = c * gj;
    g[j + 1] = -sg * gj;
    const bool finite = den < INFINITY && fabs(g[j + 1]) < INFINITY;
    G.kr[u] = finite ? j + 1 : j;  // a non-finite step is not used
    if (!finite || fabs(g[j + 1]) <= tol * G.beta[u] || b == 0.0) G.act[u] = 0;
}

// Per rhs: whether some unit of it takes more Krylov steps (the gate of the solve kernels).
__global__ void k_gm_any(DevGmres G, int nsys) {
    const int r = blockIdx.x;
    int any = 0;
    for (int q = threadIdx.x; q < nsys; q += blockDim.x) any |= G.act[r * nsys + q];
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) G.ract[r] = any;
}

// y = R^{-1} g over the kr Krylov vectors taken (back substitution; a zero pivot from a
// breakdown contributes nothing), zero beyond; y[i * U + u] as the combination expects.
__global__ void k_gm_solve(DevGmres G, int nu) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= nu) return;
    const int k = G.kr[u];
    double y[GM_M];
    for (int i = GM_M - 1; i >= 0; --i) {
        double v = 0.0;
        if (i < k) {
            v = G.g[(int64_t)u * (GM_M + 1) + i];
            for (int jj = i + 1; jj < k; ++jj) v -= G.R[((int64_t)u * GM_M + jj) * GM_M + i] * y[jj];
            const double d = G.R[((int64_t)u * GM_M + i) * GM_M + i];
            v = d != 0.0 ? v / d : 0.0;
        }
        y[i] = v;
        G.y[(int64_t)i * nu + u] = v;
    }
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- host wrappers

void launch_theta(const DevPlan& D, const double* theta, double rho, double delta, const double* rho_sys,
                  const double* delta_sys, hipStream_t s) {
    hipLaunchKernelGGL(k_init_scalars, dim3(nblocks(D.nsys, 256)), dim3(256), 0, s, D, rho, delta, rho_sys,
                       delta_sys);
    if (rho_sys || delta_sys) hipLaunchKernelGGL(k_check_shifts, dim3(nblocks(D.nsys, 256)), dim3(256), 0, s, D);
    if (D.n > 0) hipLaunchKernelGGL(k_theta, dim3(nblocks(D.n, 256)), dim3(256), 0, s, D, theta);
}

void launch_values_n(const DevPlan& D, int64_t knnz, hipStream_t s) {
    if (knnz > 0) hipLaunchKernelGGL(k_values, dim3(nblocks(knnz, 256)), dim3(256), 0, s, D, knnz);
}

void launch_knorm(const DevPlan& D, hipStream_t s) {
    if (D.N > 0) hipLaunchKernelGGL(k_rowsum, dim3(nblocks(D.N, 256)), dim3(256), 0, s, D);
    hipLaunchKernelGGL(k_knorm, dim3(D.nsys), dim3(1024), 0, s, D);
}

void launch_matrix_norms(const DevPlan& D, hipStream_t s) {
    int64_t mx = D.n > D.m ? D.n : D.m;
    if (mx > 0) hipLaunchKernelGGL(k_matrix_norms, dim3(nblocks(mx, 256)), dim3(256), 0, s, D);
}

void launch_hessian_norms(const DevPlan& D, hipStream_t s) {
    if (D.n > 0) hipLaunchKernelGGL(k_hessian_norms, dim3(nblocks(D.n, 256)), dim3(256), 0, s, D);
}

void launch_factor_step(const DevPlan& D, const Launch& L, const Task* tasks, const PivotParams& pp,
                        hipStream_t s) {
    const unsigned g = (unsigned)L.ntask;
    switch (L.kind) {
        case L_SMALL:
            if (L.maxf <= 16) hipLaunchKernelGGL(k_small<16>, dim3(g), dim3(64), 0, s, D, tasks, L.task0, pp);
            else if (L.maxf <= 32) hipLaunchKernelGGL(k_small<32>, dim3(g), dim3(64), 0, s, D, tasks, L.task0, pp);
            else hipLaunchKernelGGL(k_small<64>, dim3(g), dim3(64), 0, s, D, tasks, L.task0, pp);
            break;
        case L_ASSEMBLE:
            if (L.maxf <= 512)
                hipLaunchKernelGGL(k_assemble_w, dim3((unsigned)((L.ntask + 3) / 4)), dim3(256), (size_t)4 * L.maxf * 8,
                                   s, D, tasks, L.task0, L.ntask, L.maxf);
            else
                hipLaunchKernelGGL(k_assemble, dim3(g), dim3(256), (size_t)L.lds, s, D, tasks, L.task0);
            break;
        case L_WINDOW:
            switch (L.npg) {
                case 0: hipLaunchKernelGGL(k_window<0>, dim3(g), dim3(256), 0, s, D, tasks, L.task0, pp); break;
                case 1: hipLaunchKernelGGL(k_window<1>, dim3(g), dim3(256), 0, s, D, tasks, L.task0, pp); break;
                default: break;  // the plan uses at most one panel group per workgroup
            }
            break;
        case L_SYRK:
            hipLaunchKernelGGL(k_syrk, dim3((unsigned)(L.ntask + L.nfin)), dim3(256), 0, s, D, tasks, L.task0, pp,
                               L.ntask, L.fin0);
            break;
        case L_SYRK128: {
            // mixed precision: the tasks of fronts of order >= f_mix (the first nmix) in FP32
            const int64_t nf = pp.mixed ? L.nmix : 0;
            if (nf > 0) hipLaunchKernelGGL(k_syrk128f, dim3((unsigned)nf), dim3(256), 0, s, D, tasks, L.task0);
            if (L.ntask - nf + L.nfin > 0)
                hipLaunchKernelGGL(k_syrk128, dim3((unsigned)(L.ntask - nf + L.nfin)), dim3(256), 0, s, D, tasks,
                                   L.task0 + nf, L.ntask - nf, L.fin0);
            break;
        }
        case L_FINALIZE: hipLaunchKernelGGL(k_finalize, dim3(g), dim3(256), 0, s, D, tasks, L.task0); break;
        default: break;
    }
}

int factor_stats_blocks(int64_t N) { return (int)std::max<int64_t>(1, (N + FS_PER_BLOCK - 1) / FS_PER_BLOCK); }

void launch_factor_stats(const DevPlan& D, const PivotParams& pp, double* part, hipStream_t s) {
    const int g = factor_stats_blocks(D.N);
    hipLaunchKernelGGL(k_factor_stats, dim3(g), dim3(256), 0, s, D, pp, part);
    hipLaunchKernelGGL(k_factor_stats_final, dim3(1), dim3(64), 0, s, D, (const double*)part, g);
    if (D.nsys > 1) hipLaunchKernelGGL(k_sys_inertia, dim3(D.nsys), dim3(256), 0, s, D);
}

void launch_mixed_check(const DevPlan& D, const PivotParams& pp, int64_t max_piv, hipStream_t s) {
    const int64_t n = (int64_t)D.nsys + 1;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, D.redo, n, 0);
    if (max_piv > 0)
        hipLaunchKernelGGL(k_mixed_check, dim3((unsigned)((max_piv + MC_CHUNK - 1) / MC_CHUNK), (unsigned)D.nsys),
                           dim3(256), 0, s, D, pp);
    hipLaunchKernelGGL(k_mixed_count, dim3(1), dim3(256), 0, s, D);
}

void launch_matvec(const DevPlan& D, const double* v, double* out, int nrhs, double* lsum, const int32_t* act,
                   hipStream_t s) {
    if (D.mode == 1 && D.nlong > 0)
        hipLaunchKernelGGL(k_long_cols, dim3(D.nlong, nrhs), dim3(256), 0, s, D, v, lsum, act);
    hipLaunchKernelGGL(k_matvec, dim3(nblocks(D.N, 256), nrhs), dim3(256), 0, s, D, v, out, nrhs,
                       (const double*)lsum, act);
}

void launch_dots(const DevPlan& D, const double* V, int nv, const double* w, double* out, int nrhs,
                 const int32_t* act, hipStream_t s) {
    hipLaunchKernelGGL(k_dots, dim3(nv, nrhs * D.nsys), dim3(256), 0, s, D, V, nv, w, out, nrhs, act);
}

void launch_vcombine(const DevPlan& D, const double* V, int nv, const double* h, double* w, int nrhs, bool subtract,
                     const int32_t* act, const int32_t* nvr, hipStream_t s) {
    hipLaunchKernelGGL(k_vcombine, dim3(nblocks(D.N, 256), nrhs), dim3(256), 0, s, D, V, nv, h, w, nrhs,
                       subtract ? 1 : 0, act, nvr);
}

void launch_vscale(const DevPlan& D, const double* src, const double* nrm2, double* dst, int nrhs,
                   const int32_t* act, hipStream_t s) {
    hipLaunchKernelGGL(k_vscale, dim3(nblocks(D.N, 256), nrhs), dim3(256), 0, s, D, src, nrm2, dst, nrhs, act);
}

// ---- the Krylov correction's small dense part, one thread per refinement unit
void launch_gm_start(const DevGmres& G, const int32_t* gate, int nu, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_start, dim3(nblocks(nu, 256)), dim3(256), 0, s, G, gate, nu);
}

void launch_gm_rotate(const DevGmres& G, int j, int nrhs, int nsys, double tol, hipStream_t s) {
    const int nu = nrhs * nsys;
    hipLaunchKernelGGL(k_gm_rotate, dim3(nblocks(nu, 256)), dim3(256), 0, s, G, j, nu, tol);
    hipLaunchKernelGGL(k_gm_any, dim3(nrhs), dim3(256), 0, s, G, nsys);
}

void launch_gm_gate(const DevGmres& G, int nrhs, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_any, dim3(nrhs), dim3(256), 0, s, G, nsys);
}

void launch_gm_solve(const DevGmres& G, int nu, hipStream_t s) {
    hipLaunchKernelGGL(k_gm_solve, dim3(nblocks(nu, 256)), dim3(256), 0, s, G, nu);
}

void launch_zero(double* p, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n);
}

void launch_rhs(const DevPlan& D, const DevSolve& S, const double* r7, const double* r1, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, S, r7, r1);
}

void launch_permute(const DevPlan& D, const DevSolve& S, const double* src, const int32_t* active,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, src, S.xw, active);
}

void launch_unpermute(const DevPlan& D, const DevSolve& S, double* dst, const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_unpermute, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, S.xw, dst, active);
}

void launch_solve_level(bool forward, const DevPlan& D, const DevSolve& S, const int32_t* lvl_sn_dev,
                        int64_t base, unsigned count, int32_t maxf, int32_t maxp, const int32_t* active,
                        hipStream_t s) {
    if (!count) return;
    if (maxf <= 64) {  // one wavefront per supernode
        const dim3 g((count + 3) / 4);
        const int c = (int)count;
#define QDMF_WAVE_LAUNCH(K, PM) hipLaunchKernelGGL(K<PM>, g, dim3(256), 0, s, D, S, lvl_sn_dev, base, c, active)
        if (forward) {
            if (maxp <= 8) QDMF_WAVE_LAUNCH(k_fwd_wave, 8);
            else if (maxp <= 16) QDMF_WAVE_LAUNCH(k_fwd_wave, 16);
            else if (maxp <= 32) QDMF_WAVE_LAUNCH(k_fwd_wave, 32);
            else QDMF_WAVE_LAUNCH(k_fwd_wave, 64);
        } else {
            if (maxp <= 8) QDMF_WAVE_LAUNCH(k_bwd_wave, 8);
            else if (maxp <= 16) QDMF_WAVE_LAUNCH(k_bwd_wave, 16);
            else if (maxp <= 32) QDMF_WAVE_LAUNCH(k_bwd_wave, 32);
            else QDMF_WAVE_LAUNCH(k_bwd_wave, 64);
        }
#undef QDMF_WAVE_LAUNCH
        return;
    }
    const size_t lds = (size_t)maxf * 8;
    const int v = maxp <= 8 ? 0 : maxp <= 16 ? 1 : maxp <= 32 ? 2 : 3;
#define QDMF_SOLVE_LAUNCH(K, NBM) hipLaunchKernelGGL(K<NBM>, dim3(count), dim3(256), lds, s, D, S, lvl_sn_dev, base, active)
    if (forward) {
        if (v == 0) QDMF_SOLVE_LAUNCH(k_fwd, 8);
        else if (v == 1) QDMF_SOLVE_LAUNCH(k_fwd, 16);
        else if (v == 2) QDMF_SOLVE_LAUNCH(k_fwd, 32);
        else QDMF_SOLVE_LAUNCH(k_fwd, 64);
    } else {
        if (v == 0) QDMF_SOLVE_LAUNCH(k_bwd, 8);
        else if (v == 1) QDMF_SOLVE_LAUNCH(k_bwd, 16);
        else if (v == 2) QDMF_SOLVE_LAUNCH(k_bwd, 32);
        else QDMF_SOLVE_LAUNCH(k_bwd, 64);
    }
#undef QDMF_SOLVE_LAUNCH
}

void launch_inv(const DevPlan& D, const Task* tasks, int64_t ntask, hipStream_t s) {
    if (ntask > 0) hipLaunchKernelGGL(k_inv, dim3((unsigned)ntask), dim3(64), 0, s, D, tasks);
}

void launch_big_solve(const DevPlan& D, const DevSolve& S, const SolveLaunch& L, const Task* stasks,
                      const int32_t* active, hipStream_t s) {
    const unsigned g = (unsigned)L.ntask;
    switch (L.kind) {
        case S_GATHER: hipLaunchKernelGGL(k_sgather, dim3(g), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        case S_FDIAG: hipLaunchKernelGGL(k_sfdiag, dim3(g), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        case S_FUPD: hipLaunchKernelGGL(k_sfupd, dim3(g, 4), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        case S_FFIN: hipLaunchKernelGGL(k_sffin, dim3(g), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        case S_BLOAD: hipLaunchKernelGGL(k_sbload, dim3(g), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        case S_BPART: hipLaunchKernelGGL(k_sbpart, dim3(g, SB / 64), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        case S_BDIAG: hipLaunchKernelGGL(k_sbdiag, dim3(g), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        case S_BSTORE: hipLaunchKernelGGL(k_sbstore, dim3(g), dim3(256), 0, s, D, S, stasks, L.task0, active); break;
        default: break;
    }
}

void launch_residual(const DevPlan& D, const DevSolve& S, const double* x, hipStream_t s) {
    if (D.mode == 1 && D.nlong > 0)
        hipLaunchKernelGGL(k_long_cols, dim3(D.nlong, S.nrhs), dim3(256), 0, s, D, x, S.lsum, (const int32_t*)nullptr);
    hipLaunchKernelGGL(k_residual, dim3(S.nblk, S.nrhs), dim3(256), 0, s, D, S, x);
}

void launch_berr_steps(const DevPlan& D, const DevSolve& S, int32_t phase, double target, int max_steps,
                       hipStream_t s) {
    if (D.nsys == 1) {
        hipLaunchKernelGGL(k_berr_cw, dim3(S.nblk, S.nrhs), dim3(256), 0, s, D, S, phase);
        hipLaunchKernelGGL(k_berr_fin, dim3(S.nrhs), dim3(256), 0, s, D, S, phase, target, max_steps);
        return;
    }
    hipLaunchKernelGGL(k_berr, dim3(D.nsys, S.nrhs), dim3(1024), 0, s, D, S, phase, target, max_steps);
    hipLaunchKernelGGL(k_any_active, dim3(S.nrhs), dim3(256), 0, s, D, S);
}

void launch_refine_begin(const DevPlan& D, const DevSolve& S, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_begin, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, S);
}

void launch_refine_update(const DevPlan& D, const DevSolve& S, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_update, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, S);
}

void launch_recover(const DevPlan& D, const DevSolve& S, const double* r7, double* dx, double* dy,
                    hipStream_t s) {
    int64_t mx = D.n > D.m ? D.n : D.m;
    hipLaunchKernelGGL(k_recover, dim3(nblocks(mx, 256), S.nrhs), dim3(256), 0, s, D, S, r7, dx, dy);
}

}  // namespace qdmf
