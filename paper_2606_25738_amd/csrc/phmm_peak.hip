// Vector-ALU FMA rate microbenchmark (calibration of the roofline peak).
//
// Every lane runs 8 independent FMA chains; with enough wavefronts per SIMD
// the VALU issue rate, not latency, bounds the run.  Packed FP32 forms are
// disabled at build time, so the FP32 figure is the scalar FMA rate.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "phmm.h"

namespace {

template <typename R>
__global__ __launch_bounds__(256) void fma_chains(R* out, int iters, R a, R b)
{
    R x0 = (R)threadIdx.x * (R)1e-3, x1 = x0 + (R)1, x2 = x0 + (R)2, x3 = x0 + (R)3;
    R x4 = x0 + (R)4, x5 = x0 + (R)5, x6 = x0 + (R)6, x7 = x0 + (R)7;
    for (int i = 0; i < iters; ++i) {
        x0 = __builtin_fma(x0, a, b); x1 = __builtin_fma(x1, a, b);
        x2 = __builtin_fma(x2, a, b); x3 = __builtin_fma(x3, a, b);
        x4 = __builtin_fma(x4, a, b); x5 = __builtin_fma(x5, a, b);
        x6 = __builtin_fma(x6, a, b); x7 = __builtin_fma(x7, a, b);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

template <>
__global__ __launch_bounds__(256) void fma_chains<float>(float* out, int iters, float a, float b)
{
    float x0 = (float)threadIdx.x * 1e-3f, x1 = x0 + 1.f, x2 = x0 + 2.f, x3 = x0 + 3.f;
    float x4 = x0 + 4.f, x5 = x0 + 5.f, x6 = x0 + 6.f, x7 = x0 + 7.f;
    for (int i = 0; i < iters; ++i) {
        x0 = __builtin_fmaf(x0, a, b); x1 = __builtin_fmaf(x1, a, b);
        x2 = __builtin_fmaf(x2, a, b); x3 = __builtin_fmaf(x3, a, b);
        x4 = __builtin_fmaf(x4, a, b); x5 = __builtin_fmaf(x5, a, b);
        x6 = __builtin_fmaf(x6, a, b); x7 = __builtin_fmaf(x7, a, b);
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

template <typename R>
double run(int cus, int iters)
{
    const int blocks = cus * 16, threads = 256;
    R* out = nullptr;
    if (hipMalloc(&out, sizeof(R) * blocks * threads) != hipSuccess) return -1.0;
    hipEvent_t e0, e1;
    double tflops = -1.0;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        hipLaunchKernelGGL(fma_chains<R>, dim3(blocks), dim3(threads), 0, 0, out, iters / 8,
                           (R)0.9999999, (R)1e-7);
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(fma_chains<R>, dim3(blocks), dim3(threads), 0, 0, out, iters,
                           (R)0.9999999, (R)1e-7);
        (void)hipEventRecord(e1, 0);
        float ms = 0.f;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
            ms > 0.f)
            tflops = 2.0 * 8.0 * (double)iters * blocks * threads / (ms * 1e-3) / 1e12;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    (void)hipFree(out);
    return tflops;
}

}  // namespace

extern "C" int phmm_vector_peak(int device, double* fp32_tflops, double* fp64_tflops)
{
    if (!fp32_tflops || !fp64_tflops) return PHMM_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return PHMM_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PHMM_EDEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return PHMM_EDEVICE;
    *fp32_tflops = run<float>(prop.multiProcessorCount, 1 << 14);
    *fp64_tflops = run<double>(prop.multiProcessorCount, 1 << 13);
    return (*fp32_tflops > 0 && *fp64_tflops > 0) ? PHMM_OK : PHMM_EDEVICE;
}
