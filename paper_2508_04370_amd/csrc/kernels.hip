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

#include <cmath>
#include <cstdint>

#include "device.hpp"

namespace qdmf {

namespace {

constexpr int LDT = 65;  // leading dimension of LDS tiles (doubles), odd to spread banks

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline void wave_argmax(double v, int idx, double& bv, int& bi) {
    // maximum value, lowest index among equal maxima
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double ov = __shfl_xor(v, off);
        int oi = __shfl_xor(idx, off);
        if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
        }
    }
    bv = v;
    bi = idx;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// LDS state of the one-wave pivot kernel.  T holds a full symmetric fr x fr matrix
// (fr <= 64), T[i][j] at j*LDT + i; the first nbw columns are the pivot window.
struct PivShared {
    double T[64 * LDT];
    double sh[64];  // static shift of the row (-rho primal, +delta dual)
    double w0[64], w1[64];
    double d[64], doff[64], ed[64];
    int sg[64];     // expected pivot sign
    int pm[64];     // original position now at this position
    int pt[64], fl[64], zs[64];
};

__device__ void sym_swap(PivShared& S, int fr, int a, int b, int lane) {
    if (a == b) return;
    if (lane < fr) {  // rows a and b
        double t = S.T[lane * LDT + a];
        S.T[lane * LDT + a] = S.T[lane * LDT + b];
        S.T[lane * LDT + b] = t;
    }
    __syncthreads();
    if (lane < fr) {  // columns a and b
        double t = S.T[a * LDT + lane];
        S.T[a * LDT + lane] = S.T[b * LDT + lane];
        S.T[b * LDT + lane] = t;
    }
    if (lane == 0) {
        int ts = S.sg[a]; S.sg[a] = S.sg[b]; S.sg[b] = ts;
        double tz = S.sh[a]; S.sh[a] = S.sh[b]; S.sh[b] = tz;
        int tp = S.pm[a]; S.pm[a] = S.pm[b]; S.pm[b] = tp;
    }
    __syncthreads();
}

// Partial LDL^T of the window [0, nbw) of the fr x fr matrix in S.T; rows [nbw, fr) are
// eliminated too (right-looking).  One wavefront (blockDim.x == 64).
__device__ void factor_window(PivShared& S, int fr, int nbw, double knorm, const PivotParams& pp,
                              int lane) {
    const double tiny = pp.eps_lift * knorm;  // delta * ||M||_1 of the lift test
    const double alpha = pp.alpha;
    int k = 0;
    while (k < nbw) {
        if (pp.presort) {  // largest |diagonal| of the window to position k
            double v = (lane >= k && lane < nbw) ? fabs(S.T[lane * LDT + lane]) : -1.0;
            double bv;
            int q;
            wave_argmax(v, lane, bv, q);
            sym_swap(S, fr, k, q, lane);
        }
        double gp;
        int r;
        {
            double v = (lane > k && lane < nbw) ? fabs(S.T[k * LDT + lane]) : -1.0;
            wave_argmax(v, lane, gp, r);
            if (!(gp > 0.0)) {
                gp = 0.0;
                r = -1;
            }
        }
        const double akk = fabs(S.T[k * LDT + k]);
        int two = 0, lifted = 0;
        double fkk_before = S.T[k * LDT + k];
        if (fmax(akk, gp) <= tiny) {
            lifted = 1;
        } else if (akk >= alpha * gp) {
            // 1x1 at k
        } else {
            double v2 = (lane >= k && lane < nbw && lane != r) ? fabs(S.T[r * LDT + lane]) : -1.0;
            double gr = wave_max(v2);
            if (gr < 0.0) gr = 0.0;
            if (akk * gr >= alpha * gp * gp) {
                // 1x1 at k
            } else if (fabs(S.T[r * LDT + r]) >= alpha * gr) {
                sym_swap(S, fr, k, r, lane);
                fkk_before = S.T[k * LDT + k];
            } else {
                sym_swap(S, fr, k + 1, r, lane);
                two = 1;
            }
        }
        if (two) {
            const double a = S.T[k * LDT + k] + S.sh[k];
            const double b = S.T[k * LDT + k + 1];
            const double c = S.T[(k + 1) * LDT + k + 1] + S.sh[k + 1];
            const double det = a * c - b * b;
            if (det == 0.0) {
                two = 0;
                fkk_before = S.T[k * LDT + k];
                lifted = 1;
            } else {
                const bool act = lane >= k + 2 && lane < fr;
                double u0 = 0.0, u1 = 0.0, l0 = 0.0, l1 = 0.0;
                if (act) {
                    u0 = S.T[k * LDT + lane];
                    u1 = S.T[(k + 1) * LDT + lane];
                    l0 = (u0 * c - u1 * b) / det;
                    l1 = (u1 * a - u0 * b) / det;
                }
                S.w0[lane] = l0;
                S.w1[lane] = l1;
                __syncthreads();
                if (act)
                    for (int j = k + 2; j < fr; ++j) S.T[j * LDT + lane] -= u0 * S.w0[j] + u1 * S.w1[j];
                __syncthreads();
                if (act) {
                    S.T[k * LDT + lane] = l0;
                    S.T[(k + 1) * LDT + lane] = l1;
                }
                if (lane == 0) {
                    S.T[k * LDT + k + 1] = 0.0;
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
        if (lifted && lane == 0) S.T[k * LDT + k] = S.sg[k] * tiny;
        __syncthreads();
        double dk = S.T[k * LDT + k] + S.sh[k];  // static regularisation after the pivot
        const int sgk = S.sg[k];
        double q = -1.0;
        int zz = 0;
        if (lane > k && lane < nbw && S.sg[lane] == sgk) {
            double den = fabs(S.T[lane * LDT + lane] + S.sh[lane]);
            if (den == 0.0) zz = 1;
            else {
                double fjk = S.T[k * LDT + lane];
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
        const bool act = lane > k && lane < fr;
        double li = 0.0;
        if (act) {
            li = S.T[k * LDT + lane] / dk;
            for (int j = k + 1; j < fr; ++j) S.T[j * LDT + lane] -= li * S.T[k * LDT + j];
        }
        __syncthreads();
        if (act) S.T[k * LDT + lane] = li;
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

__device__ inline void init_signs(PivShared& S, const DevPlan& D, const int32_t* rows, int fr,
                                  int lane) {
    const double rho = D.sc->rho, delta = D.sc->delta;
    if (lane < fr) {
        const bool pr = D.primal_new[rows[lane]] != 0;
        S.sg[lane] = pr ? -1 : 1;
        S.sh[lane] = pr ? -rho : delta;
        S.pm[lane] = lane;
    }
}

__device__ inline void store_pivots(const PivShared& S, const DevPlan& D, int pos0, int k0, int nbw,
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

// Small fronts (f <= 64): assembly of original entries and children's contribution blocks
// straight into LDS, then the whole partial factorisation there.
__global__ __launch_bounds__(64) void k_small(DevPlan D, const Task* tasks, int64_t t0, PivotParams pp) {
    __shared__ PivShared S;
    const int lane = threadIdx.x;
    const int s = tasks[t0 + blockIdx.x].s;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    double* F = D.front + D.sn_off[s];
    const int32_t* rows = D.rows + D.sn_rowptr[s];
    for (int j = 0; j < 64; ++j) S.T[j * LDT + lane] = 0.0;
    __syncthreads();
    for (int c = 0; c < p; ++c) {
        const int64_t e1 = D.kcol_ptr[c0 + c + 1];
        for (int64_t e = D.kcol_ptr[c0 + c] + lane; e < e1; e += 64) {
            const int r = D.kloc[e];
            const double v = D.kval[e];
            S.T[c * LDT + r] = v;
            S.T[r * LDT + c] = v;
        }
    }
    __syncthreads();
    for (int q = D.ch_ptr[s]; q < D.ch_ptr[s + 1]; ++q) {  // children in ascending order
        const int ch = D.ch[q];
        const int cp = D.sn_p[ch], cb = D.sn_f[ch] - cp, cld = D.sn_ld[ch];
        const double* CF = D.front + D.sn_off[ch];
        const int32_t* rel = D.rel + D.rel_ptr[ch];
        for (int b = 0; b < cb; ++b) {
            const int rb = rel[b];
            for (int a = b + lane; a < cb; a += 64) {
                const int ra = rel[a];
                const double v = CF[(cp + a) + (int64_t)(cp + b) * cld];
                S.T[rb * LDT + ra] += v;
                if (a != b) S.T[ra * LDT + rb] += v;
            }
        }
        __syncthreads();
    }
    init_signs(S, D, rows, f, lane);
    __syncthreads();
    factor_window(S, f, p, D.sc->knorm, pp, lane);
    for (int j = 0; j < f; ++j)
        if (lane >= j && lane < f) F[lane + (int64_t)j * ld] = S.T[j * LDT + lane];
    store_pivots(S, D, c0, 0, p, lane);
}

// Large fronts: one workgroup per front column.  The column is summed in LDS from the
// original entries and, children in ascending order, the children's contribution-block
// columns that map onto it (the parent pulls; no atomics), then written once.
__global__ __launch_bounds__(256) void k_assemble(DevPlan D, const Task* tasks, int64_t t0) {
    extern __shared__ double buf[];
    const Task t = tasks[t0 + blockIdx.x];
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
    for (int q = D.ch_ptr[s]; q < D.ch_ptr[s + 1]; ++q) {
        const int ch = D.ch[q];
        const int cp = D.sn_p[ch], cb = D.sn_f[ch] - cp, cld = D.sn_ld[ch];
        const int32_t* rel = D.rel + D.rel_ptr[ch];
        int lo = 0, hi = cb;  // rel is increasing: find the CB column mapped to j
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (rel[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        if (lo < cb && rel[lo] == j) {
            const double* col = D.front + D.sn_off[ch] + (int64_t)(cp + lo) * cld + cp;
            for (int a = lo + tid; a < cb; a += 256) buf[rel[a] - j] += col[a];
        }
        __syncthreads();
    }
    double* out = D.front + D.sn_off[s] + (int64_t)j * ld + j;
    for (int i = tid; i < nr; i += 256) out[i] = buf[i];
}

// Diagonal block of window [k0, k0+nbw) of a large front.
__global__ __launch_bounds__(64) void k_diag(DevPlan D, const Task* tasks, int64_t t0, PivotParams pp) {
    __shared__ PivShared S;
    const int lane = threadIdx.x;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, k0 = t.k0;
    const int p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int nbw = min(NB, p - k0);
    double* F = D.front + D.sn_off[s] + k0 + (int64_t)k0 * ld;
    for (int j = 0; j < nbw; ++j)
        if (lane >= j && lane < nbw) {
            const double v = F[lane + (int64_t)j * ld];
            S.T[j * LDT + lane] = v;
            S.T[lane * LDT + j] = v;
        }
    init_signs(S, D, D.rows + D.sn_rowptr[s] + k0, nbw, lane);
    __syncthreads();
    factor_window(S, nbw, nbw, D.sc->knorm, pp, lane);
    for (int j = 0; j < nbw; ++j)
        if (lane >= j && lane < nbw) F[lane + (int64_t)j * ld] = S.T[j * LDT + lane];
    store_pivots(S, D, c0 + k0, k0, nbw, lane);
}

// Rows below the window: apply the window's column permutation, then
// L21 = B_P L11^{-T} D^{-1}, by forward substitution per row (one row per lane).
__global__ __launch_bounds__(64) void k_panel(DevPlan D, const Task* tasks, int64_t t0) {
    __shared__ double L[64 * LDT];
    __shared__ double Wl[64 * 64];
    __shared__ double dd[64], od[64];
    __shared__ int pt[64], pm[64];
    const int lane = threadIdx.x;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, k0 = t.k0, chunk = t.a;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int k1 = min(k0 + NB, p), nbw = k1 - k0;
    double* F = D.front + D.sn_off[s];
    for (int j = 0; j < 64; ++j) {
        double v = 0.0;
        if (j < nbw && lane > j && lane < nbw) v = F[(k0 + lane) + (int64_t)(k0 + j) * ld];
        L[j * LDT + lane] = v;
    }
    if (lane < nbw) {
        dd[lane] = D.dval[c0 + k0 + lane];
        od[lane] = D.doff[c0 + k0 + lane];
        pt[lane] = D.ptype[c0 + k0 + lane];
        pm[lane] = D.lperm[c0 + k0 + lane] - k0;
    } else {
        dd[lane] = 1.0;
        od[lane] = 0.0;
        pt[lane] = 0;
        pm[lane] = 0;
    }
    __syncthreads();
    const int r = k1 + chunk * 64 + lane;
    const bool act = r < f;
    // each lane's row vector lives in its own LDS column: Wl[k*64 + lane]
    for (int j = 0; j < nbw; ++j) Wl[j * 64 + lane] = act ? F[r + (int64_t)(k0 + pm[j]) * ld] : 0.0;
    // w = b L11^{-T}: column-oriented forward substitution (L11 unit lower)
    for (int j = 0; j + 1 < nbw; ++j) {
        const double wj = Wl[j * 64 + lane];
        for (int k = j + 1; k < nbw; ++k) Wl[k * 64 + lane] -= L[j * LDT + k] * wj;
    }
    // L21 = w D^{-1}, 1x1 and 2x2 blocks
    if (act) {
        for (int k = 0; k < nbw; ++k) {
            const int ty = pt[k];
            const double wk = Wl[k * 64 + lane];
            double v;
            if (ty == 0) {
                v = wk / dd[k];
            } else if (ty == 1) {
                const double a = dd[k], b = od[k], c = dd[k + 1];
                v = (wk * c - Wl[(k + 1) * 64 + lane] * b) / (a * c - b * b);
            } else {
                const double a = dd[k - 1], b = od[k - 1], c = dd[k];
                v = (wk * a - Wl[(k - 1) * 64 + lane] * b) / (a * c - b * b);
            }
            F[r + (int64_t)(k0 + k) * ld] = v;
        }
    }
}

// Trailing update of one 64 x 64 lower tile: C -= L21 W^T with W = L21 D, on MFMA.
// The tile is computed transposed (C^T = W L21^T) so that each group of 16 lanes stores
// 16 consecutive rows of one column.  T = double: FP64 MFMA 16x16x4; T = float: operands
// rounded to FP32, FP32 MFMA with FP32 accumulation, result subtracted in FP64.
template <typename T>
__device__ void syrk_tile(double* F, int ld, int f, int k0, int nbw, int R0, int C0,
                          const double* dd, const double* od, const int* pt, T* As, T* Bs) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 64 * 64; idx += 256) {
        const int kk = idx >> 6, r = idx & 63;
        const int row = R0 + r, col = C0 + r;
        double a = 0.0, b = 0.0;
        if (kk < nbw) {
            if (row < f) a = F[row + (int64_t)(k0 + kk) * ld];
            if (col < f) {
                const double* cr = F + col + (int64_t)k0 * ld;
                const int ty = pt[kk];
                if (ty == 0) b = cr[(int64_t)kk * ld] * dd[kk];
                else if (ty == 1) b = cr[(int64_t)kk * ld] * dd[kk] + cr[(int64_t)(kk + 1) * ld] * od[kk];
                else b = cr[(int64_t)(kk - 1) * ld] * od[kk - 1] + cr[(int64_t)kk * ld] * dd[kk];
            }
        }
        As[r * LDT + kk] = (T)a;
        Bs[r * LDT + kk] = (T)b;
    }
    __syncthreads();
    const int wv = tid >> 6, l = tid & 63;
    const int wc = (wv >> 1) * 32, wr = (wv & 1) * 32;
    const int li = l & 15, lk = l >> 4;
    if constexpr (sizeof(T) == 8) {
        d4 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        for (int kk = 0; kk < 64; kk += 4) {
            double a0 = Bs[(wc + li) * LDT + kk + lk];
            double a1 = Bs[(wc + 16 + li) * LDT + kk + lk];
            double b0 = As[(wr + li) * LDT + kk + lk];
            double b1 = As[(wr + 16 + li) * LDT + kk + lk];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // f64 16x16x4 output: element (lk + 4v, li) of the 16 x 16 block
                    const int col = C0 + wc + i * 16 + lk + 4 * v;
                    const int row = R0 + wr + j * 16 + li;
                    if (row < f && col < f && row >= col) F[row + (int64_t)col * ld] -= acc[i][j][v];
                }
    } else {
        f4 acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        for (int kk = 0; kk < 64; kk += 4) {
            float a0 = Bs[(wc + li) * LDT + kk + lk];
            float a1 = Bs[(wc + 16 + li) * LDT + kk + lk];
            float b0 = As[(wr + li) * LDT + kk + lk];
            float b1 = As[(wr + 16 + li) * LDT + kk + lk];
            acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    // f32 16x16x4 output: element (4 lk + v, li) of the 16 x 16 block
                    const int col = C0 + wc + i * 16 + 4 * lk + v;
                    const int row = R0 + wr + j * 16 + li;
                    if (row < f && col < f && row >= col) F[row + (int64_t)col * ld] -= (double)acc[i][j][v];
                }
    }
}

__global__ __launch_bounds__(256) void k_syrk(DevPlan D, const Task* tasks, int64_t t0, PivotParams pp) {
    __shared__ double As[64 * LDT];
    __shared__ double Bs[64 * LDT];
    __shared__ double dd[64], od[64];
    __shared__ int pt[64];
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, k0 = t.k0;
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int k1 = min(k0 + NB, p), nbw = k1 - k0;
    const int tid = threadIdx.x;
    if (tid < 64) {
        if (tid < nbw) {
            dd[tid] = D.dval[c0 + k0 + tid];
            od[tid] = D.doff[c0 + k0 + tid];
            pt[tid] = D.ptype[c0 + k0 + tid];
        } else {
            dd[tid] = 0.0;
            od[tid] = 0.0;
            pt[tid] = 0;
        }
    }
    __syncthreads();
    double* F = D.front + D.sn_off[s];
    const int R0 = k1 + 64 * t.a, C0 = k1 + 64 * t.b;
    if (pp.mixed && f >= pp.f_mix)
        syrk_tile<float>(F, ld, f, k0, nbw, R0, C0, dd, od, pt, (float*)As, (float*)Bs);
    else
        syrk_tile<double>(F, ld, f, k0, nbw, R0, C0, dd, od, pt, As, Bs);
}

// After all windows of a front: permute the rows of each earlier L column that lie in a
// later window, as that window's pivot swaps require.
__global__ __launch_bounds__(64) void k_rowswap(DevPlan D, const Task* tasks, int64_t t0) {
    const int lane = threadIdx.x;
    const Task t = tasks[t0 + blockIdx.x];
    const int s = t.s, col0 = t.k0;
    const int p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const int nwin = (p + NB - 1) / NB;
    const int jend = min(col0 + 64, (nwin - 1) * NB);
    double* F = D.front + D.sn_off[s];
    for (int j = col0; j < jend; ++j) {
        for (int w = j / NB + 1; w < nwin; ++w) {
            const int k0 = w * NB, nbw = min(NB, p - k0);
            double v = 0.0;
            if (lane < nbw) v = F[k0 + (D.lperm[c0 + k0 + lane] - k0) + (int64_t)j * ld];
            __syncthreads();
            if (lane < nbw) F[k0 + lane + (int64_t)j * ld] = v;
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------- values of K

__global__ void k_init_scalars(DevPlan D, double rho, double delta) {
    D.sc->rho = rho;
    D.sc->delta = delta;
    D.sc->bad_theta = 0;
    D.sc->knorm = 0.0;
}

// AS: dinv = 1/Theta (diagonal -(Theta^{-1}) of equation (augsys));
// NE: dinv = theta~ = 1/(1/Theta + rho) (equation (regul_matrix)).
__global__ void k_theta(DevPlan D, const double* theta) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= D.n) return;
    const double th = theta[j];
    if (!(th > 0.0) || !isfinite(th)) atomicOr(&D.sc->bad_theta, 1);
    if (D.mode == 1) D.dinv[j] = 1.0 / th;
    else D.dinv[j] = 1.0 / (1.0 / th + D.sc->rho);
}

// Values of lower(K) in analyse order.  NE: K_ik = sum_j (A_ij theta~_j) A_kj over the
// shared columns j in ascending order (fixed order, no atomics).
__global__ void k_values(DevPlan D, int64_t knnz) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= knnz) return;
    if (D.mode == 1) {
        const int64_t src = D.ksrc[e];
        double v;
        if (src >= 0) v = D.aval[src];
        else if (src == KSRC_ZERO) v = 0.0;
        else v = -D.dinv[-1 - src];
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
    const double rho = D.sc->rho, delta = D.sc->delta;
    double s;
    if (D.mode == 1) {
        if (i < D.n) s = (D.dinv[i] + rho) + D.colabs[i];
        else s = D.rowabs[i - D.n] + delta;
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

__global__ __launch_bounds__(1024) void k_knorm(DevPlan D) {
    __shared__ double red[1024];
    double m = 0.0;
    for (int i = threadIdx.x; i < D.N; i += 1024) m = fmax(m, D.rowsum[i]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) D.sc->knorm = red[0];
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

// Inertia and regularisation counts over all pivot positions (fixed-order reduction).
__global__ __launch_bounds__(1024) void k_factor_stats(DevPlan D, PivotParams pp) {
    __shared__ int64_t ri[8][1024];
    __shared__ double rd[1024];
    int64_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double me = 0.0;
    int big = 0;
    const double thr = pp.tau_big * D.sc->knorm;
    for (int k = threadIdx.x; k < D.N; k += 1024) {
        const int ty = D.ptype[k];
        if (ty == 0) {
            const double d = D.dval[k];
            if (d < 0) c[0]++;
            else if (d > 0) c[1]++;
            else c[2]++;
        } else if (ty == 1) {
            c[3]++;
            const double a = D.dval[k], b = D.doff[k], cc = D.dval[k + 1];
            const double det = a * cc - b * b;
            if (det < 0) { c[0]++; c[1]++; }
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
        big |= e > thr;
    }
    for (int q = 0; q < 8; ++q) ri[q][threadIdx.x] = c[q];
    rd[threadIdx.x] = big ? -fmax(me, 0.0) - 1.0 : me;  // sign carries the flag
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            for (int q = 0; q < 8; ++q) ri[q][threadIdx.x] += ri[q][threadIdx.x + w];
            const double a = rd[threadIdx.x], b = rd[threadIdx.x + w];
            const bool fa = a < 0, fb = b < 0;
            const double ma = fa ? -a - 1.0 : a, mb = fb ? -b - 1.0 : b;
            const double mm = fmax(ma, mb);
            rd[threadIdx.x] = (fa || fb) ? -mm - 1.0 : mm;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        DevStats* st = D.st;
        st->nneg = ri[0][0];
        st->npos = ri[1][0];
        st->nzero = ri[2][0];
        st->n2x2 = ri[3][0];
        st->nlift = ri[4][0];
        st->nprop3 = ri[5][0];
        st->nsign = ri[6][0];
        st->nzskip = ri[7][0];
        const double v = rd[0];
        st->large_reg = v < 0;
        st->max_edyn = v < 0 ? -v - 1.0 : v;
        st->bad_theta = D.sc->bad_theta;
    }
}

// ---------------------------------------------------------------- solve kernels

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

// Forward substitution with unit L and the D solve for the supernodes of one level.  The
// parent gathers its children's contribution vectors (ascending order, no atomics).
__global__ __launch_bounds__(256) void k_fwd(DevPlan D, DevSolve S, const int32_t* lvl_sn, int64_t base,
                                             const int32_t* active) {
    extern __shared__ double y[];
    const int s = lvl_sn[base + blockIdx.x];
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const double* F = D.front + D.sn_off[s];
    const int tid = threadIdx.x;
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        double* xw = S.xw + (int64_t)r * D.N;
        for (int i = tid; i < f; i += 256) y[i] = i < p ? xw[c0 + D.lperm[c0 + i]] : 0.0;
        __syncthreads();
        for (int q = D.ch_ptr[s]; q < D.ch_ptr[s + 1]; ++q) {
            const int ch = D.ch[q];
            const int cb = D.sn_f[ch] - D.sn_p[ch];
            const int32_t* rel = D.rel + D.rel_ptr[ch];
            const double* u = S.ub + D.ub_off[ch] + (int64_t)r * D.ub_total;
            // the child->parent map addresses pre-pivot rows; pivot rows moved in factorisation
            for (int a = tid; a < cb; a += 256) {
                const int t = rel[a];
                y[t < p ? D.lpinv[c0 + t] : t] += u[a];
            }
            __syncthreads();
        }
        for (int k0 = 0; k0 < p; k0 += 64) {
            const int k1 = min(k0 + 64, p);
            if (tid < 64) {
                const int row = k0 + tid;
                for (int k = k0; k < k1; ++k) {
                    const double z = y[k];
                    if (row > k && row < k1) y[row] -= F[row + (int64_t)k * ld] * z;
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
            for (int i = k1 + tid; i < f; i += 256) {
                double acc = y[i];
                for (int k = k0; k < k1; ++k) acc -= F[i + (int64_t)k * ld] * y[k];
                y[i] = acc;
            }
            __syncthreads();
        }
        double* u = S.ub + D.ub_off[s] + (int64_t)r * D.ub_total;
        for (int i = p + tid; i < f; i += 256) u[i - p] = y[i];
        for (int k = tid; k < p; k += 256) {  // block-diagonal D
            const int ty = D.ptype[c0 + k];
            double v;
            if (ty == 0) v = y[k] / D.dval[c0 + k];
            else if (ty == 1) {
                const double a = D.dval[c0 + k], b = D.doff[c0 + k], c = D.dval[c0 + k + 1];
                v = (c * y[k] - b * y[k + 1]) / (a * c - b * b);
            } else {
                const double a = D.dval[c0 + k - 1], b = D.doff[c0 + k - 1], c = D.dval[c0 + k];
                v = (a * y[k] - b * y[k - 1]) / (a * c - b * b);
            }
            xw[c0 + D.lperm[c0 + k]] = v;
        }
        __syncthreads();
    }
}

// Backward substitution with L^T for the supernodes of one level (ancestors done).
__global__ __launch_bounds__(256) void k_bwd(DevPlan D, DevSolve S, const int32_t* lvl_sn, int64_t base,
                                             const int32_t* active) {
    extern __shared__ double y[];
    const int s = lvl_sn[base + blockIdx.x];
    const int f = D.sn_f[s], p = D.sn_p[s], c0 = D.sn_ptr[s], ld = D.sn_ld[s];
    const double* F = D.front + D.sn_off[s];
    const int32_t* rows = D.rows + D.sn_rowptr[s];
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    for (int r = 0; r < S.nrhs; ++r) {
        if (active && !active[r]) continue;
        double* xw = S.xw + (int64_t)r * D.N;
        for (int i = tid; i < f; i += 256) y[i] = i < p ? xw[c0 + D.lperm[c0 + i]] : xw[rows[i]];
        __syncthreads();
        const int nblk = (p + 63) / 64;
        for (int bk = nblk - 1; bk >= 0; --bk) {
            const int k0 = bk * 64, k1 = min(k0 + 64, p);
            for (int k = k0 + wv; k < k1; k += 4) {  // rows below the block
                double part = 0.0;
                for (int i = k1 + lane; i < f; i += 64) part += F[i + (int64_t)k * ld] * y[i];
                part = wave_sum_d(part);
                if (lane == 0) y[k] -= part;
            }
            __syncthreads();
            if (tid < 64) {
                for (int k = k1 - 1; k >= k0; --k) {
                    const int i = k + 1 + lane;
                    double part = (i < k1) ? F[i + (int64_t)k * ld] * y[i] : 0.0;
                    part = wave_sum_d(part);
                    if (lane == 0) y[k] -= part;
                    __builtin_amdgcn_wave_barrier();
                }
            }
            __syncthreads();
        }
        for (int k = tid; k < p; k += 256) xw[c0 + D.lperm[c0 + k]] = y[k];
        __syncthreads();
    }
}

// r = b - K_static x and (|K||x|)_i in original numbering, from A, Theta, rho, delta
// (AS) or from the K values (NE); per-block maxima of |r|, |x|, |b|.
__global__ __launch_bounds__(256) void k_residual(DevPlan D, DevSolve S, const double* xin) {
    __shared__ double red[3][256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    const double* x = xin + (int64_t)r * D.N;
    const double* b = S.b + (int64_t)r * D.N;
    double ar = 0.0, ax = 0.0, ab = 0.0;
    if (i < D.N) {
        const double rho = D.sc->rho, delta = D.sc->delta;
        double kx = 0.0, akx = 0.0;
        if (D.mode == 1) {
            if (i < D.n) {
                const double dj = -(D.dinv[i] + rho);
                kx = dj * x[i];
                akx = fabs(dj) * fabs(x[i]);
                for (int64_t e = D.acp[i]; e < D.acp[i + 1]; ++e) {
                    const double a = D.aval[e], xv = x[D.n + D.ari[e]];
                    kx += a * xv;
                    akx += fabs(a) * fabs(xv);
                }
            } else {
                const int row = i - D.n;
                for (int64_t q = D.arp[row]; q < D.arp[row + 1]; ++q) {
                    const int32_t e = D.are[q];
                    const double a = D.aval[e], xv = x[D.acol[e]];
                    kx += a * xv;
                    akx += fabs(a) * fabs(xv);
                }
                kx += delta * x[i];
                akx += delta * fabs(x[i]);
            }
        } else {
            for (int64_t q = D.krs_ptr[i]; q < D.krs_ptr[i + 1]; ++q) {
                const int o = D.krs_other[q];
                double v = D.kval[D.krs_ent[q]];
                if (o == i) v += delta;
                kx += v * x[o];
                akx += fabs(v) * fabs(x[o]);
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
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x < 3) S.part[(int64_t)r * 3 * S.nblk + threadIdx.x * S.nblk + blockIdx.x] = red[threadIdx.x][0];
}

// Backward errors (normwise in the infinity norm; componentwise with the small-denominator
// substitution of Arioli, Demmel and Duff) and the refinement decision for each rhs.
// phase 0: after the first solve; phase 1: after a refinement step.
__global__ __launch_bounds__(1024) void k_berr(DevPlan D, DevSolve S, int phase, double target, int max_steps) {
    __shared__ double red[1024];
    __shared__ double sh_rmax, sh_xmax, sh_bmax;
    const int r = blockIdx.x;
    if (phase == 1 && !S.active[r]) return;
    const double* part = S.part + (int64_t)r * 3 * S.nblk;
    for (int q = 0; q < 3; ++q) {
        double m = 0.0;
        for (int i = threadIdx.x; i < S.nblk; i += 1024) m = fmax(m, part[q * S.nblk + i]);
        red[threadIdx.x] = m;
        __syncthreads();
        for (int w = 512; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (q == 0) sh_rmax = red[0];
            else if (q == 1) sh_xmax = red[0];
            else sh_bmax = red[0];
        }
        __syncthreads();
    }
    const double xmax = sh_xmax;
    const double u = 1.1102230246251565e-16;
    const double* rr = S.r + (int64_t)r * D.N;
    const double* akx = S.d + (int64_t)r * D.N;
    const double* b = S.b + (int64_t)r * D.N;
    double cm = 0.0;
    for (int i = threadIdx.x; i < D.N; i += 1024) {
        double den = akx[i] + fabs(b[i]);
        if (den <= 1000.0 * D.N * u * (D.rowsum[i] * xmax + fabs(b[i]))) den = akx[i] + xmax * D.rowsum[i];
        const double c = den > 0 ? fabs(rr[i]) / den : (rr[i] == 0 ? 0.0 : INFINITY);
        cm = fmax(cm, c);
    }
    red[threadIdx.x] = cm;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double cw = red[0];
    const double den = D.sc->knorm * xmax + sh_bmax;
    const double nw = den > 0 ? sh_rmax / den : (sh_rmax == 0 ? 0.0 : INFINITY);
    double* be = S.berr + 4 * r;
    __shared__ int restore;
    if (threadIdx.x == 0) {
        restore = 0;
        if (phase == 0) {
            be[0] = nw;
            be[1] = cw;
            be[2] = nw;
            S.steps[r] = 0;
            S.active[r] = (nw > target && max_steps > 0) ? 1 : 0;
        } else {
            const double prev = be[0];
            if (!(nw < prev)) {  // no improvement: keep the previous iterate
                restore = 1;
                S.active[r] = 0;
                S.steps[r] += 1;
            } else {
                S.steps[r] += 1;
                const bool stagnating = nw > 0.5 * prev;
                be[0] = nw;
                be[1] = cw;
                S.active[r] = (!stagnating && nw > target && S.steps[r] < max_steps) ? 1 : 0;
            }
        }
    }
    __syncthreads();
    if (restore) {
        double* x = S.x + (int64_t)r * D.N;
        const double* xb = S.xbak + (int64_t)r * D.N;
        for (int i = threadIdx.x; i < D.N; i += 1024) x[i] = xb[i];
    }
}

__global__ void k_refine_begin(DevPlan D, DevSolve S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N || !S.active[r]) return;
    S.xbak[i + (int64_t)r * D.N] = S.x[i + (int64_t)r * D.N];
}

__global__ void k_refine_update(DevPlan D, DevSolve S) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= D.N || !S.active[r]) return;
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

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- host wrappers

void launch_theta(const DevPlan& D, const double* theta, double rho, double delta, hipStream_t s) {
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(1), 0, s, D, rho, delta);
    if (D.n > 0) hipLaunchKernelGGL(k_theta, dim3(nblocks(D.n, 256)), dim3(256), 0, s, D, theta);
}

void launch_values_n(const DevPlan& D, int64_t knnz, hipStream_t s) {
    if (knnz > 0) hipLaunchKernelGGL(k_values, dim3(nblocks(knnz, 256)), dim3(256), 0, s, D, knnz);
}

void launch_knorm(const DevPlan& D, hipStream_t s) {
    if (D.N > 0) hipLaunchKernelGGL(k_rowsum, dim3(nblocks(D.N, 256)), dim3(256), 0, s, D);
    hipLaunchKernelGGL(k_knorm, dim3(1), dim3(1024), 0, s, D);
}

void launch_matrix_norms(const DevPlan& D, hipStream_t s) {
    int64_t mx = D.n > D.m ? D.n : D.m;
    if (mx > 0) hipLaunchKernelGGL(k_matrix_norms, dim3(nblocks(mx, 256)), dim3(256), 0, s, D);
}

void launch_factor_step(const DevPlan& D, const Launch& L, const Task* tasks, const PivotParams& pp,
                        hipStream_t s) {
    const unsigned g = (unsigned)L.ntask;
    switch (L.kind) {
        case L_SMALL: hipLaunchKernelGGL(k_small, dim3(g), dim3(64), 0, s, D, tasks, L.task0, pp); break;
        case L_ASSEMBLE:
            hipLaunchKernelGGL(k_assemble, dim3(g), dim3(256), (size_t)L.lds, s, D, tasks, L.task0);
            break;
        case L_DIAG: hipLaunchKernelGGL(k_diag, dim3(g), dim3(64), 0, s, D, tasks, L.task0, pp); break;
        case L_PANEL: hipLaunchKernelGGL(k_panel, dim3(g), dim3(64), 0, s, D, tasks, L.task0); break;
        case L_SYRK: hipLaunchKernelGGL(k_syrk, dim3(g), dim3(256), 0, s, D, tasks, L.task0, pp); break;
        case L_ROWSWAP: hipLaunchKernelGGL(k_rowswap, dim3(g), dim3(64), 0, s, D, tasks, L.task0); break;
        default: break;
    }
}

void launch_factor_stats(const DevPlan& D, const PivotParams& pp, hipStream_t s) {
    hipLaunchKernelGGL(k_factor_stats, dim3(1), dim3(1024), 0, s, D, pp);
}

void launch_zero(double* p, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_zero, dim3(nblocks(n, 256)), dim3(256), 0, s, p, n);
}

void launch_rhs(const DevPlan& D, const DevSolve& S, const double* r7, const double* r1, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, S, r7, r1);
}

void launch_ldlt_solve_levels(const DevPlan& D, const DevSolve& S, const int32_t* lvl_sn_dev,
                              const int64_t* lvl_ptr, int nlevels, const int32_t* maxf_lvl,
                              const double* src, double* dst, const int32_t* active, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, src, S.xw, active);
    for (int l = 0; l < nlevels; ++l) {
        const unsigned g = (unsigned)(lvl_ptr[l + 1] - lvl_ptr[l]);
        if (g) hipLaunchKernelGGL(k_fwd, dim3(g), dim3(256), (size_t)maxf_lvl[l] * 8, s, D, S, lvl_sn_dev, lvl_ptr[l], active);
    }
    for (int l = nlevels - 1; l >= 0; --l) {
        const unsigned g = (unsigned)(lvl_ptr[l + 1] - lvl_ptr[l]);
        if (g) hipLaunchKernelGGL(k_bwd, dim3(g), dim3(256), (size_t)maxf_lvl[l] * 8, s, D, S, lvl_sn_dev, lvl_ptr[l], active);
    }
    hipLaunchKernelGGL(k_unpermute, dim3(nblocks(D.N, 256), S.nrhs), dim3(256), 0, s, D, S.xw, dst, active);
}

void launch_residual(const DevPlan& D, const DevSolve& S, const double* x, hipStream_t s) {
    hipLaunchKernelGGL(k_residual, dim3(S.nblk, S.nrhs), dim3(256), 0, s, D, S, x);
}

void launch_berr_steps(const DevPlan& D, const DevSolve& S, int32_t phase, double target, int max_steps,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_berr, dim3(S.nrhs), dim3(1024), 0, s, D, S, phase, target, max_steps);
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
