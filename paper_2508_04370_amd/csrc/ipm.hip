// Device kernels of the interior point driver (Section 3 of the paper) for the LP with bounds
// of Section 2: min c^T x subject to A x = b, x - x^l = l, x + x^u = u, x^l, x^u >= 0, with
// every l finite and u finite or +inf; for a quadratic program the objective gains
// x^T Q x / 2 (Q from the handle) and the dual residual +Q x.  The kernels compute the
// residuals and the scalars of the termination test, Theta, the right-hand sides of the
// predictor and of the centrality correctors, the recovery of a direction from its dx, step
// lengths to the boundary, the complementarity at a trial point, and the update.  Reductions
// are per-block partials combined in a fixed order by one workgroup, so every run gives the
// same bits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.hpp"

namespace qdmf {
namespace {

constexpr int IPM_T = 256;

__device__ inline double block_reduce(double v, double* red, bool is_max) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = IPM_T / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            red[threadIdx.x] = is_max ? fmax(red[threadIdx.x], red[threadIdx.x + w]) : red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline double lower(const double* l, int i) { return l ? l[i] : 0.0; }
__device__ inline bool has_upper(const double* u, int i) { return u && isfinite(u[i]); }

// Start point: x = l + 1, or the midpoint of [l, u] where u - l < 2; x^l = x - l,
// x^u = u - x; z^l = 1, z^u = 1 where u is finite; y = 0.  Per block: the number of bad
// bounds (l not finite, u NaN or -inf, or finite u <= l) and of finite u.
__global__ __launch_bounds__(IPM_T) void k_ipm_start(const double* l, const double* u, IpmVec p, int n, int m,
                                                     double* part) {
    __shared__ double red[IPM_T];
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    double bad = 0.0, nu = 0.0;
    if (i < n) {
        const double li = lower(l, i);
        const bool hu = has_upper(u, i);
        if (!isfinite(li) || (u && (isnan(u[i]) || u[i] == -INFINITY)) || (hu && !(u[i] > li))) bad = 1.0;
        double x = li + 1.0;
        if (hu && u[i] - li < 2.0) x = 0.5 * (li + u[i]);
        p.x[i] = x;
        p.xl[i] = x - li;
        p.xu[i] = hu ? u[i] - x : 0.0;
        p.zl[i] = 1.0;
        p.zu[i] = hu ? 1.0 : 0.0;
        nu = hu ? 1.0 : 0.0;
    }
    if (i < m) p.y[i] = 0.0;
    const double sb = block_reduce(bad, red, false), su = block_reduce(nu, red, false);
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * IPM_PART + 0] = sb;
        part[(int64_t)blockIdx.x * IPM_PART + 1] = su;
    }
}

// Residuals of Section 3: r1 = b - A x (rows); r2 = l - x + x^l, r3 = u - x - x^u (0 where
// u is infinite), r4 = c - A^T y - z^l + z^u (+ Q x) (columns).  Per block, the quantities
//   0 max|r1|  1 max|r4|  2 sum c x  3 sum b y  4 sum x^l z^l + x^u z^u  5 max|b|  6 max|c|
//   7 max|r2|  8 max|r3|  9 sum l z^l  10 sum u z^u (finite u)  11 max|l|  12 max|u| (finite u)
//   13 sum x (Q x)
constexpr int RESID_Q = 14;
constexpr unsigned RESID_MAX_MASK = (1u << 0) | (1u << 1) | (1u << 5) | (1u << 6) | (1u << 7) | (1u << 8) |
                                    (1u << 11) | (1u << 12);

__global__ __launch_bounds__(IPM_T) void k_ipm_resid(DevPlan D, IpmVec p, const double* b, const double* c,
                                                     const double* l, const double* u, double* r1, double* r2,
                                                     double* r3, double* r4, double* part) {
    __shared__ double red[IPM_T];
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    double v[RESID_Q];
    for (int q = 0; q < RESID_Q; ++q) v[q] = 0.0;
    if (i < D.m) {
        double ax = 0.0;
        for (int64_t q = D.arp[i]; q < D.arp[i + 1]; ++q) {
            const int32_t e = D.are[q];
            ax += D.aval[e] * p.x[D.acol[e]];
        }
        const double r = b[i] - ax;
        r1[i] = r;
        v[0] = fabs(r);
        v[3] = b[i] * p.y[i];
        v[5] = fabs(b[i]);
    }
    if (i < D.n) {
        double aty = 0.0;
        for (int64_t e = D.acp[i]; e < D.acp[i + 1]; ++e) aty += D.aval[e] * p.y[D.ari[e]];
        double qx = 0.0;
        if (D.has_q)
            for (int64_t e = D.qfcp[i]; e < D.qfcp[i + 1]; ++e) qx += D.qval[D.qfsrc[e]] * p.x[D.qfri[e]];
        const double ra = D.has_q ? (c[i] - aty - p.zl[i] + p.zu[i]) + qx : c[i] - aty - p.zl[i] + p.zu[i];
        r4[i] = ra;
        const double li = lower(l, i);
        const bool hu = has_upper(u, i);
        const double rb = li - p.x[i] + p.xl[i];
        const double rc = hu ? u[i] - p.x[i] - p.xu[i] : 0.0;
        r2[i] = rb;
        r3[i] = rc;
        v[1] = fabs(ra);
        v[2] = c[i] * p.x[i];
        v[4] = p.xl[i] * p.zl[i] + (hu ? p.xu[i] * p.zu[i] : 0.0);
        v[6] = fabs(c[i]);
        v[7] = fabs(rb);
        v[8] = fabs(rc);
        v[9] = li * p.zl[i];
        v[10] = hu ? u[i] * p.zu[i] : 0.0;
        v[11] = fabs(li);
        v[12] = hu ? fabs(u[i]) : 0.0;
        v[13] = p.x[i] * qx;
    }
    for (int q = 0; q < RESID_Q; ++q) {
        const double s = block_reduce(v[q], red, (RESID_MAX_MASK >> q) & 1u);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * IPM_PART + q] = s;
    }
}

// Combines nq quantities of nblk per-block partials (stride IPM_PART): maxima for the entries
// of max_mask, sums otherwise, in block order; out[q].
__global__ __launch_bounds__(IPM_T) void k_ipm_combine(const double* part, int nblk, int nq, unsigned max_mask,
                                                       double* out) {
    __shared__ double red[IPM_T];
    for (int q = 0; q < nq; ++q) {
        const bool mx = (max_mask >> q) & 1u;
        double v = mx ? -INFINITY : 0.0;
        // each thread combines a contiguous run of blocks in order, then the runs in order
        const int per = (nblk + IPM_T - 1) / IPM_T;
        const int g0 = threadIdx.x * per, g1 = min(nblk, g0 + per);
        for (int g = g0; g < g1; ++g)
            v = mx ? fmax(v, part[(int64_t)g * IPM_PART + q]) : v + part[(int64_t)g * IPM_PART + q];
        red[threadIdx.x] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = red[0];
            for (int k = 1; k < IPM_T; ++k) t = mx ? fmax(t, red[k]) : t + red[k];
            out[q] = t;
        }
        __syncthreads();
    }
}

// Theta = 1 / (z^l / x^l + z^u / x^u)
__global__ void k_ipm_theta(IpmVec p, const double* u, double* theta, int n) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i >= n) return;
    double t = p.zl[i] / p.xl[i];
    if (has_upper(u, i)) t += p.zu[i] / p.xu[i];
    theta[i] = 1.0 / t;
}

// Complementarity target of a centrality corrector for one product: v at the trial point is
// moved into [bmin smu, bmax smu]; the move is at least -bmax smu.
__device__ inline double corr_target(double xv, double dxv, double zv, double dzv, double tp, double td, double smu,
                                     double bmin, double bmax) {
    const double v = (xv + tp * dxv) * (zv + td * dzv);
    const double t = fmin(fmax(v, bmin * smu), bmax * smu) - v;
    return fmax(t, -bmax * smu);
}

// mode 0 (predictor, sigma = 0): r5 = -X^l z^l, r6 = -X^u z^u,
//   r7 = r4 - (X^l)^-1 (r5 + Z^l r2) + (X^u)^-1 (r6 - Z^u r3).
// mode 1 (centrality corrector, r1 = r2 = r3 = r4 = 0): r5, r6 the targets at the trial point
//   p + (tp, td) d; r7 = -(X^l)^-1 r5 + (X^u)^-1 r6.
__global__ void k_ipm_rhs(int mode, IpmVec p, IpmVec d, const double* u, const double* r2, const double* r3,
                          const double* r4, double smu, double tp, double td, double bmin, double bmax, double* r5,
                          double* r6, double* r7, int n) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i >= n) return;
    const bool hu = has_upper(u, i);
    double t5, t6 = 0.0, s7;
    if (mode == 0) {
        t5 = -p.xl[i] * p.zl[i];
        s7 = r4[i] - (t5 + p.zl[i] * r2[i]) / p.xl[i];
        if (hu) {
            t6 = -p.xu[i] * p.zu[i];
            s7 += (t6 - p.zu[i] * r3[i]) / p.xu[i];
        }
    } else {
        t5 = corr_target(p.xl[i], d.xl[i], p.zl[i], d.zl[i], tp, td, smu, bmin, bmax);
        s7 = -t5 / p.xl[i];
        if (hu) {
            t6 = corr_target(p.xu[i], d.xu[i], p.zu[i], d.zu[i], tp, td, smu, bmin, bmax);
            s7 += t6 / p.xu[i];
        }
    }
    r5[i] = t5;
    r6[i] = t6;
    r7[i] = s7;
}

// dx^l = dx - r2, dx^u = r3 - dx, dz^l = (X^l)^-1 (r5 - Z^l dx^l), dz^u = (X^u)^-1 (r6 - Z^u dx^u)
__global__ void k_ipm_recover(IpmVec p, IpmVec d, const double* u, const double* r2, const double* r3,
                              const double* r5, const double* r6, int n) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i >= n) return;
    const double dx = d.x[i];
    const double dxl = r2 ? dx - r2[i] : dx;
    d.xl[i] = dxl;
    d.zl[i] = (r5[i] - p.zl[i] * dxl) / p.xl[i];
    if (has_upper(u, i)) {
        const double dxu = r3 ? r3[i] - dx : -dx;
        d.xu[i] = dxu;
        d.zu[i] = (r6[i] - p.zu[i] * dxu) / p.xu[i];
    } else {
        d.xu[i] = 0.0;
        d.zu[i] = 0.0;
    }
}

__global__ void k_ipm_add(IpmVec a, IpmVec b, IpmVec o, int n, int m) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < n) {
        o.x[i] = a.x[i] + b.x[i];
        o.xl[i] = a.xl[i] + b.xl[i];
        o.xu[i] = a.xu[i] + b.xu[i];
        o.zl[i] = a.zl[i] + b.zl[i];
        o.zu[i] = a.zu[i] + b.zu[i];
    }
    if (i < m) o.y[i] = a.y[i] + b.y[i];
}

// per block: the largest steps in (0, 1] keeping x^l, x^u (primal) and z^l, z^u (dual)
// nonnegative, written negated so that one maximum reduction gives the minima
__global__ __launch_bounds__(IPM_T) void k_ipm_step(IpmVec p, IpmVec d, const double* u, double* part, int n) {
    __shared__ double red[IPM_T];
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    double ap = 1.0, ad = 1.0;
    if (i < n) {
        if (d.xl[i] < 0) ap = fmin(ap, -p.xl[i] / d.xl[i]);
        if (d.zl[i] < 0) ad = fmin(ad, -p.zl[i] / d.zl[i]);
        if (has_upper(u, i)) {
            if (d.xu[i] < 0) ap = fmin(ap, -p.xu[i] / d.xu[i]);
            if (d.zu[i] < 0) ad = fmin(ad, -p.zu[i] / d.zu[i]);
        }
    }
    const double mp = block_reduce(-ap, red, true), md = block_reduce(-ad, red, true);
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * IPM_PART + 0] = mp;
        part[(int64_t)blockIdx.x * IPM_PART + 1] = md;
    }
}

// per block: sum of (x^l + ap dx^l)(z^l + ad dz^l) + (x^u + ap dx^u)(z^u + ad dz^u)
__global__ __launch_bounds__(IPM_T) void k_ipm_comp(IpmVec p, IpmVec d, const double* u, double ap, double ad,
                                                    double* part, int n) {
    __shared__ double red[IPM_T];
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    double v = 0.0;
    if (i < n) {
        v = (p.xl[i] + ap * d.xl[i]) * (p.zl[i] + ad * d.zl[i]);
        if (has_upper(u, i)) v += (p.xu[i] + ap * d.xu[i]) * (p.zu[i] + ad * d.zu[i]);
    }
    const double s = block_reduce(v, red, false);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * IPM_PART] = s;
}

__global__ void k_ipm_update(IpmVec p, IpmVec d, double sp, double sd, int n, int m) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < n) {
        p.x[i] += sp * d.x[i];
        p.xl[i] += sp * d.xl[i];
        p.xu[i] += sp * d.xu[i];
        p.zl[i] += sd * d.zl[i];
        p.zu[i] += sd * d.zu[i];
    }
    if (i < m) p.y[i] += sd * d.y[i];
}

__global__ void k_ipm_fill(double* v, double a, int len) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < len) v[i] = a;
}

unsigned nb(int64_t len) { return (unsigned)std::max<int64_t>(1, (len + IPM_T - 1) / IPM_T); }

}  // namespace

int ipm_blocks(int64_t len) { return (int)nb(len); }

void ipm_start(const double* l, const double* u, IpmVec p, int n, int m, double* part, double* out, hipStream_t s) {
    const unsigned g = nb(std::max(n, m));
    hipLaunchKernelGGL(k_ipm_start, dim3(g), dim3(IPM_T), 0, s, l, u, p, n, m, part);
    hipLaunchKernelGGL(k_ipm_combine, dim3(1), dim3(IPM_T), 0, s, part, (int)g, 2, 0x0u, out);
}

void ipm_resid(const DevPlan& D, IpmVec p, const double* b, const double* c, const double* l, const double* u,
               double* r1, double* r2, double* r3, double* r4, double* part, double* out, hipStream_t s) {
    const unsigned g = nb(std::max(D.n, D.m));
    hipLaunchKernelGGL(k_ipm_resid, dim3(g), dim3(IPM_T), 0, s, D, p, b, c, l, u, r1, r2, r3, r4, part);
    hipLaunchKernelGGL(k_ipm_combine, dim3(1), dim3(IPM_T), 0, s, part, (int)g, RESID_Q, RESID_MAX_MASK, out);
}

void ipm_theta(IpmVec p, const double* u, double* theta, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_theta, dim3(nb(n)), dim3(IPM_T), 0, s, p, u, theta, n);
}

void ipm_rhs(int mode, IpmVec p, IpmVec d, const double* u, const double* r2, const double* r3, const double* r4,
             double smu, double tp, double td, double bmin, double bmax, double* r5, double* r6, double* r7, int n,
             hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_rhs, dim3(nb(n)), dim3(IPM_T), 0, s, mode, p, d, u, r2, r3, r4, smu, tp, td, bmin, bmax,
                       r5, r6, r7, n);
}

void ipm_recover(IpmVec p, IpmVec d, const double* u, const double* r2, const double* r3, const double* r5,
                 const double* r6, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_recover, dim3(nb(n)), dim3(IPM_T), 0, s, p, d, u, r2, r3, r5, r6, n);
}

void ipm_add(IpmVec a, IpmVec b, IpmVec out, int n, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_add, dim3(nb(std::max(n, m))), dim3(IPM_T), 0, s, a, b, out, n, m);
}

void ipm_step(IpmVec p, IpmVec d, const double* u, double* part, double* out, int n, hipStream_t s) {
    const unsigned g = nb(n);
    hipLaunchKernelGGL(k_ipm_step, dim3(g), dim3(IPM_T), 0, s, p, d, u, part, n);
    hipLaunchKernelGGL(k_ipm_combine, dim3(1), dim3(IPM_T), 0, s, part, (int)g, 2, 0x3u, out);
}

void ipm_comp(IpmVec p, IpmVec d, const double* u, double ap, double ad, double* part, double* out, int n,
              hipStream_t s) {
    const unsigned g = nb(n);
    hipLaunchKernelGGL(k_ipm_comp, dim3(g), dim3(IPM_T), 0, s, p, d, u, ap, ad, part, n);
    hipLaunchKernelGGL(k_ipm_combine, dim3(1), dim3(IPM_T), 0, s, part, (int)g, 1, 0x0u, out);
}

void ipm_update(IpmVec p, IpmVec d, double sp, double sd, int n, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_update, dim3(nb(std::max(n, m))), dim3(IPM_T), 0, s, p, d, sp, sd, n, m);
}

void ipm_fill(double* v, double a, int len, hipStream_t s) {
    if (len > 0) hipLaunchKernelGGL(k_ipm_fill, dim3(nb(len)), dim3(IPM_T), 0, s, v, a, len);
}

}  // namespace qdmf
