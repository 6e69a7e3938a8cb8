// Device kernels of the interior point driver (Section 3 of the paper): residuals and their
// norms, Theta, the complementarity right-hand sides of the predictor and of the centrality
// correctors, the recovery of dz, step lengths to the boundary, and the update.  LP form:
// min c^T x, A x = b, x >= 0 (lower bounds at zero, none above).  Reductions are per-block
// partials combined in a fixed order by one workgroup, so every run gives the same bits.
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

// r1 = b - A x (rows), r4 = c - A^T y - z (columns); per block: max|r1|, max|r4|, sum c x,
// sum b y, sum x z, max|b|, max|c|.
__global__ __launch_bounds__(IPM_T) void k_ipm_resid(DevPlan D, const double* x, const double* y, const double* z,
                                                     const double* b, const double* c, double* r1, double* r4,
                                                     double* part) {
    __shared__ double red[IPM_T];
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    if (i < D.m) {
        double ax = 0.0;
        for (int64_t q = D.arp[i]; q < D.arp[i + 1]; ++q) {
            const int32_t e = D.are[q];
            ax += D.aval[e] * x[D.acol[e]];
        }
        const double r = b[i] - ax;
        r1[i] = r;
        v[0] = fabs(r);
        v[3] = b[i] * y[i];
        v[5] = fabs(b[i]);
    }
    if (i < D.n) {
        double aty = 0.0;
        for (int64_t e = D.acp[i]; e < D.acp[i + 1]; ++e) aty += D.aval[e] * y[D.ari[e]];
        const double r = c[i] - aty - z[i];
        r4[i] = r;
        v[1] = fabs(r);
        v[2] = c[i] * x[i];
        v[4] = x[i] * z[i];
        v[6] = fabs(c[i]);
    }
    for (int q = 0; q < 7; ++q) {
        const bool mx = q == 0 || q == 1 || q == 5 || q == 6;
        const double s = block_reduce(v[q], red, mx);
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 8 + q] = s;
    }
}

// Combines nq quantities of nblk per-block partials (stride 8): maxima for the entries of
// max_mask, sums otherwise, in block order; out[q].
__global__ __launch_bounds__(IPM_T) void k_ipm_combine(const double* part, int nblk, int nq, unsigned max_mask,
                                                       double* out) {
    __shared__ double red[IPM_T];
    for (int q = 0; q < nq; ++q) {
        const bool mx = (max_mask >> q) & 1u;
        double v = mx ? -INFINITY : 0.0;
        // each thread combines a contiguous run of blocks in order, then the runs in order
        const int per = (nblk + IPM_T - 1) / IPM_T;
        const int g0 = threadIdx.x * per, g1 = min(nblk, g0 + per);
        for (int g = g0; g < g1; ++g) v = mx ? fmax(v, part[(int64_t)g * 8 + q]) : v + part[(int64_t)g * 8 + q];
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

__global__ void k_ipm_theta(const double* x, const double* z, double* theta, int n) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < n) theta[i] = x[i] / z[i];
}

// mode 0 (predictor, sigma = 0): r5 = -x z, r7 = r4 - r5 / x.
// mode 1 (centrality corrector): v = (x + tp dx)(z + td dz); r5 = clip(v, bmin smu,
// bmax smu) - v, at least -bmax smu; r7 = -r5 / x (r1 = r4 = 0).
__global__ void k_ipm_r5r7(int mode, const double* x, const double* z, const double* r4, const double* dx,
                           const double* dz, double smu, double tp, double td, double bmin, double bmax, double* r5,
                           double* r7, int n) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i >= n) return;
    double t;
    if (mode == 0) {
        t = -x[i] * z[i];
        r7[i] = r4[i] - t / x[i];
    } else {
        const double v = (x[i] + tp * dx[i]) * (z[i] + td * dz[i]);
        t = fmin(fmax(v, bmin * smu), bmax * smu) - v;
        t = fmax(t, -bmax * smu);
        r7[i] = -t / x[i];
    }
    r5[i] = t;
}

// dz = (r5 - z dx) / x
__global__ void k_ipm_dz(const double* x, const double* z, const double* r5, const double* dx, double* dz, int n) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < n) dz[i] = (r5[i] - z[i] * dx[i]) / x[i];
}

__global__ void k_ipm_add(const double* a, const double* b, double* out, int len) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < len) out[i] = a[i] + b[i];
}

// per block: min over dx < 0 of -x/dx, and over dz < 0 of -z/dz (1 where none)
__global__ __launch_bounds__(IPM_T) void k_ipm_step(const double* x, const double* dx, const double* z,
                                                    const double* dz, double* part, int n) {
    __shared__ double red[IPM_T];
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    double ap = 1.0, ad = 1.0;
    if (i < n) {
        if (dx[i] < 0) ap = fmin(1.0, -x[i] / dx[i]);
        if (dz[i] < 0) ad = fmin(1.0, -z[i] / dz[i]);
    }
    // minima through maxima of the negated values
    const double mp = block_reduce(-ap, red, true), md = block_reduce(-ad, red, true);
    if (threadIdx.x == 0) {
        part[(int64_t)blockIdx.x * 8 + 0] = mp;
        part[(int64_t)blockIdx.x * 8 + 1] = md;
    }
}

// per block: sum of (x + ap dx)(z + ad dz)
__global__ __launch_bounds__(IPM_T) void k_ipm_comp(const double* x, const double* dx, const double* z,
                                                    const double* dz, double ap, double ad, double* part, int n) {
    __shared__ double red[IPM_T];
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    const double v = i < n ? (x[i] + ap * dx[i]) * (z[i] + ad * dz[i]) : 0.0;
    const double s = block_reduce(v, red, false);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 8] = s;
}

__global__ void k_ipm_update(double* x, double* y, double* z, const double* dx, const double* dy, const double* dz,
                             double sp, double sd, int n, int m) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < n) {
        x[i] += sp * dx[i];
        z[i] += sd * dz[i];
    }
    if (i < m) y[i] += sd * dy[i];
}

__global__ void k_ipm_fill(double* v, double a, int len) {
    const int i = blockIdx.x * IPM_T + threadIdx.x;
    if (i < len) v[i] = a;
}

unsigned nb(int64_t len) { return (unsigned)std::max<int64_t>(1, (len + IPM_T - 1) / IPM_T); }

}  // namespace

int ipm_blocks(int64_t len) { return (int)nb(len); }

void ipm_resid(const DevPlan& D, const double* x, const double* y, const double* z, const double* b,
               const double* c, double* r1, double* r4, double* part, double* out, hipStream_t s) {
    const unsigned g = nb(std::max(D.n, D.m));
    hipLaunchKernelGGL(k_ipm_resid, dim3(g), dim3(IPM_T), 0, s, D, x, y, z, b, c, r1, r4, part);
    hipLaunchKernelGGL(k_ipm_combine, dim3(1), dim3(IPM_T), 0, s, part, (int)g, 7, 0x63u, out);
}

void ipm_theta(const double* x, const double* z, double* theta, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_theta, dim3(nb(n)), dim3(IPM_T), 0, s, x, z, theta, n);
}

void ipm_r5r7(int mode, const double* x, const double* z, const double* r4, const double* dx, const double* dz,
              double smu, double tp, double td, double bmin, double bmax, double* r5, double* r7, int n,
              hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_r5r7, dim3(nb(n)), dim3(IPM_T), 0, s, mode, x, z, r4, dx, dz, smu, tp, td, bmin, bmax,
                       r5, r7, n);
}

void ipm_dz(const double* x, const double* z, const double* r5, const double* dx, double* dz, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_dz, dim3(nb(n)), dim3(IPM_T), 0, s, x, z, r5, dx, dz, n);
}

void ipm_add(const double* a, const double* b, double* out, int len, hipStream_t s) {
    if (len > 0) hipLaunchKernelGGL(k_ipm_add, dim3(nb(len)), dim3(IPM_T), 0, s, a, b, out, len);
}

void ipm_step(const double* x, const double* dx, const double* z, const double* dz, double* part, double* out,
              int n, hipStream_t s) {
    const unsigned g = nb(n);
    hipLaunchKernelGGL(k_ipm_step, dim3(g), dim3(IPM_T), 0, s, x, dx, z, dz, part, n);
    hipLaunchKernelGGL(k_ipm_combine, dim3(1), dim3(IPM_T), 0, s, part, (int)g, 2, 0x3u, out);
}

void ipm_comp(const double* x, const double* dx, const double* z, const double* dz, double ap, double ad,
              double* part, double* out, int n, hipStream_t s) {
    const unsigned g = nb(n);
    hipLaunchKernelGGL(k_ipm_comp, dim3(g), dim3(IPM_T), 0, s, x, dx, z, dz, ap, ad, part, n);
    hipLaunchKernelGGL(k_ipm_combine, dim3(1), dim3(IPM_T), 0, s, part, (int)g, 1, 0x0u, out);
}

void ipm_update(double* x, double* y, double* z, const double* dx, const double* dy, const double* dz, double sp,
                double sd, int n, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_ipm_update, dim3(nb(std::max(n, m))), dim3(IPM_T), 0, s, x, y, z, dx, dy, dz, sp, sd, n, m);
}

void ipm_fill(double* v, double a, int len, hipStream_t s) {
    if (len > 0) hipLaunchKernelGGL(k_ipm_fill, dim3(nb(len)), dim3(IPM_T), 0, s, v, a, len);
}

}  // namespace qdmf
