// Calibration kernels: the vector-ALU FMA rate (the roofline peak) and a
// plain device copy of known size (the reference that scales the HBM traffic
// counters of a profile).
//
// Every lane runs 16 independent FMA chains with all three operands in VGPRs
// (an operand read from an SGPR halves the FP32 issue rate); with enough
// wavefronts per SIMD the VALU issue rate, not latency, bounds the run.
// Packed FP32 forms are disabled at build time, so the FP32 figure is the
// scalar FMA rate.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "phmm.h"

namespace {

template <typename R>
__device__ __forceinline__ R fmaT(R a, R b, R c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float fmaT<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// 16 independent FMA chains per lane.
template <typename R>
__global__ __launch_bounds__(256) void fma_chains(R* out, int iters, R a, R b)
{
    R x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = (R)threadIdx.x * (R)1e-3 + (R)q;
    R av = a, bv = b;
    asm volatile("" : "+v"(av), "+v"(bv));  // keep the multiplier and addend in VGPRs
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int q = 0; q < 16; ++q) x[q] = fmaT(x[q], av, bv);
    }
    R s = (R)0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += x[q];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <typename R>
double run(int cus, int iters)
{
    const int blocks = cus * 8, threads = 256;
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
            tflops = 2.0 * 16.0 * (double)iters * blocks * threads / (ms * 1e-3) / 1e12;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    (void)hipFree(out);
    return tflops;
}

// Plain copy, 16 bytes per lane per step, grid-stride.
__global__ __launch_bounds__(256) void copy_calib_kernel(const uint4* __restrict__ src,
                                                         uint4* __restrict__ dst, uint64_t n16)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

}  // namespace

extern "C" int phmm_copy_calib(const void* src, void* dst, uint64_t bytes, void* stream)
{
    if (!src || !dst || (bytes & 15u) != 0 || ((uintptr_t)src & 15u) != 0 ||
        ((uintptr_t)dst & 15u) != 0)
        return PHMM_EINVAL;
    if (bytes == 0) return PHMM_OK;
    const uint64_t n16 = bytes / 16;
    uint64_t blocks = (n16 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(copy_calib_kernel, dim3((unsigned)blocks), dim3(256), 0,
                       static_cast<hipStream_t>(stream), static_cast<const uint4*>(src),
                       static_cast<uint4*>(dst), n16);
    return hipGetLastError() == hipSuccess ? PHMM_OK : PHMM_EDEVICE;
}

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
