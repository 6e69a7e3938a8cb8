// Measured peaks of the units the kernels run on, for the roofline fractions: the FP64 and
// FP32 16x16x4 matrix instructions the trailing update uses, dependent-free FP64 vector FMAs,
// and a streaming device copy for HBM.  Each probe is timed with HIP events on the given
// stream; the best of a few repetitions is kept.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/qdmf.h"

namespace {

typedef double pd4 __attribute__((ext_vector_type(4)));
typedef float pf4 __attribute__((ext_vector_type(4)));

constexpr int PROBE_WGS = 2048;  // eight four-wave workgroups per compute unit
constexpr int MFMA_ITERS = 2048, VALU_ITERS = 1024;

// four independent accumulation chains per wave keep the matrix pipe busy
__global__ __launch_bounds__(256) void k_peak_mfma_f64(double* out, int iters) {
    const double a = 1.0 + 1e-9 * threadIdx.x, b = 1.0 - 1e-9 * threadIdx.x;
    pd4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
    }
    out[blockIdx.x * 256 + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

__global__ __launch_bounds__(256) void k_peak_mfma_f32(float* out, int iters) {
    const float a = 1.0f + 1e-6f * threadIdx.x, b = 1.0f - 1e-6f * threadIdx.x;
    pf4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, b, c3, 0, 0, 0);
    }
    out[blockIdx.x * 256 + threadIdx.x] = c0[0] + c1[1] + c2[2] + c3[3];
}

// eight independent FMA chains per thread
__global__ __launch_bounds__(256) void k_peak_valu_f64(double* out, int iters) {
    double x[8];
    const double m = 1.0 - 1e-12 * threadIdx.x, p = 1e-12;
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = 1.0 + u * 1e-3;
    for (int i = 0; i < iters; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r)
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = fma(x[u], m, p);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += x[u];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// dst = src, 16 bytes per thread and trip
__global__ __launch_bounds__(256) void k_peak_copy(const double2* src, double2* dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

template <typename F>
double best_ms(hipStream_t s, int reps, F&& launch, bool& ok) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        ok = false;
        return 0.0;
    }
    double best = 1e30;
    for (int r = 0; r < reps + 1; ++r) {  // the first run is a warm-up
        (void)hipEventRecord(e0, s);
        launch();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) ok = false;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) ok = false;
        if (r > 0) best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

}  // namespace

extern "C" int qdmf_peak_probe(int device, void* hip_stream, double* mfma_f64_tflops, double* mfma_f32_tflops,
                               double* valu_f64_tflops, double* hbm_gbs) {
    if (hipSetDevice(device) != hipSuccess) return QDMF_ERR_HIP;
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t copy_bytes = (int64_t)1 << 30;
    const int64_t n2 = copy_bytes / 16;
    void* out = nullptr;
    void* src = nullptr;
    void* dst = nullptr;
    if (hipMalloc(&out, sizeof(double) * PROBE_WGS * 256) != hipSuccess) return QDMF_ERR_OOM;
    if (hipMalloc(&src, copy_bytes) != hipSuccess || hipMalloc(&dst, copy_bytes) != hipSuccess) {
        (void)hipFree(out);
        if (src) (void)hipFree(src);
        return QDMF_ERR_OOM;
    }
    bool ok = hipMemsetAsync(src, 0, copy_bytes, s) == hipSuccess;
    // one wave instruction of a 16x16x4 matrix product: 16 * 16 * 4 multiply-adds
    const double mfma_flops = 2.0 * 16 * 16 * 4 * 4 * (double)MFMA_ITERS * PROBE_WGS * 4;
    const double t64 = best_ms(s, 3, [&] {
        hipLaunchKernelGGL(k_peak_mfma_f64, dim3(PROBE_WGS), dim3(256), 0, s, (double*)out, MFMA_ITERS);
    }, ok);
    const double t32 = best_ms(s, 3, [&] {
        hipLaunchKernelGGL(k_peak_mfma_f32, dim3(PROBE_WGS), dim3(256), 0, s, (float*)out, MFMA_ITERS);
    }, ok);
    const double valu_flops = 2.0 * 16 * 8 * (double)VALU_ITERS * PROBE_WGS * 256;
    const double tv = best_ms(s, 3, [&] {
        hipLaunchKernelGGL(k_peak_valu_f64, dim3(PROBE_WGS), dim3(256), 0, s, (double*)out, VALU_ITERS);
    }, ok);
    const double tc = best_ms(s, 5, [&] {
        hipLaunchKernelGGL(k_peak_copy, dim3(8192), dim3(256), 0, s, (const double2*)src, (double2*)dst, n2);
    }, ok);
    (void)hipStreamSynchronize(s);
    (void)hipFree(out);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (!ok || hipGetLastError() != hipSuccess) return QDMF_ERR_HIP;
    if (mfma_f64_tflops) *mfma_f64_tflops = mfma_flops / (t64 * 1e-3) / 1e12;
    if (mfma_f32_tflops) *mfma_f32_tflops = mfma_flops / (t32 * 1e-3) / 1e12;
    if (valu_f64_tflops) *valu_f64_tflops = valu_flops / (tv * 1e-3) / 1e12;
    if (hbm_gbs) *hbm_gbs = 2.0 * (double)copy_bytes / (tc * 1e-3) / 1e9;
    return 0;
}
