// Throughput probes for the roofline denominators (include/sce_peak.h):
// independent chains of one instruction kind per wave, timed with HIP events.

#include <hip/hip_runtime.h>

#include <cstdio>

#include "sce_peak.h"

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

// The split-precision kernels' pattern: per accumulator the three products
// lo*hi, hi*lo, hi*hi of FP16 hi/lo operand pairs (hi ~0.4-0.75, lo ~1e-3,
// varying over lanes and elements), 16 accumulators per wave, 4 waves per SIMD.
constexpr int kMfmaBlocksPerCU = 4;
__global__ void __launch_bounds__(kThreads) k_mfma_f16(float *out, int iters)
{
    const int lane = threadIdx.x & 63;
    half8 h[4], l[4];
    for (int q = 0; q < 4; ++q)
        for (int i = 0; i < 8; ++i) {
            h[q][i] = (_Float16)(0.37f + 0.0131f * ((lane * 7 + i * 3 + q) % 29));
            l[q][i] = (_Float16)(0.0003f * ((lane * 5 + i * 11 + q) % 31) - 0.0045f);
        }
    f32x4 acc[16];
    for (int c = 0; c < 16; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 16; ++c) {
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(l[c & 3], h[(c + 1) & 3], acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(h[c & 3], l[(c + 1) & 3], acc[c], 0, 0, 0);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(h[c & 3], h[(c + 1) & 3], acc[c], 0, 0, 0);
        }
    }
    float r = 0.f;
    for (int c = 0; c < 16; ++c) r += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// vector FMA probes: 16 independent chains per lane, 8 waves per SIMD
constexpr int kFmaBlocksPerCU = 8;
template <typename T>
__global__ void __launch_bounds__(kThreads) k_fma(T *out, int iters)
{
    const int t = blockIdx.x * kThreads + threadIdx.x;
    T v[16];
    for (int k = 0; k < 16; ++k) v[k] = (T)(0.5 + 1e-3 * ((t * 13 + k * 7) % 97));
    const T a = (T)0.99999, c = (T)(1e-6 * (1 + (t & 15)));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = fma(v[k], a, c);
    }
    T r = 0;
    for (int k = 0; k < 16; ++k) r += v[k];
    out[t] = r;
}

int fail(hipError_t e, const char *what)
{
    std::fprintf(stderr, "sce_peak: %s: %s\n", what, hipGetErrorString(e));
    return -3;
}

#define PCHK(expr)                                \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return fail(_e, #expr); \
    } while (0)

// Launch kern(buf, iters) once to warm up and once timed; flops_per_iter_thread
// is the work of one iteration of one thread.
template <typename T>
int run(void (*kern)(T *, int), int blocks_per_cu, double flops_per_iter_thread, int iters,
        double *tflops, double *ms)
{
    int dev = 0, cus = 0;
    PCHK(hipGetDevice(&dev));
    PCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = cus * blocks_per_cu;
    T *buf = nullptr;
    PCHK(hipMalloc(&buf, (size_t)blocks * kThreads * sizeof(T)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, 0, buf, iters / 8);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, 0);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kThreads), 0, 0, buf, iters);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(e, "probe launch");
    const double flops = flops_per_iter_thread * (double)iters * blocks * kThreads;
    if (tflops) *tflops = flops / (1e-3 * t) / 1e12;
    if (ms) *ms = t;
    return 0;
}

}  // namespace

extern "C" {

int sce_peak_mfma_f16(double *tflops, double *ms)
{
    // 48 instructions of 16384 flops per iteration and wave: per thread / 64
    return run(k_mfma_f16, kMfmaBlocksPerCU, 48.0 * 16384.0 / 64.0, 6000, tflops, ms);
}

int sce_peak_fma_f32(double *tflops, double *ms)
{
    return run(k_fma<float>, kFmaBlocksPerCU, 32.0, 20000, tflops, ms);
}

int sce_peak_fma_f64(double *tflops, double *ms)
{
    return run(k_fma<double>, kFmaBlocksPerCU, 32.0, 20000, tflops, ms);
}

}  // extern "C"
