// gfx950 instruction-rate microbenchmarks: FP32 FMA, v_exp_f32, v_rcp_f32
// and their mix, plus an HBM copy.  They set the measured denominators of
// the ALU roofline of the peak-evaluation kernels.
//
// Every kernel runs kChains independent dependency chains per lane for
// `iters` iterations and stores one value per lane (so nothing is dead).
#include <hip/hip_runtime.h>

#include <cstdint>

#define UB_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kChains = 8;

__global__ void k_fma(float *out, int iters, float b, float c) {
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x * 1e-3f + j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_exp(float *out, int iters) {
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = threadIdx.x * 1e-3f + 0.1f * j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            asm volatile("v_exp_f32 %0, -%0" : "+v"(a[j]));
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_rcp(float *out, int iters) {
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = 1.5f + threadIdx.x * 1e-3f + j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            asm volatile("v_rcp_f32 %0, -%0" : "+v"(a[j]));
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// One v_rcp_f32 and `nf` FMAs per chain step (nf in 1..4).
template <int NF>
__global__ void k_mix(float *out, int iters, float b, float c) {
    float a[kChains], r[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
        a[j] = threadIdx.x * 1e-3f + j;
        r[j] = 1.5f + j;
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) {
            asm volatile("v_rcp_f32 %0, -%0" : "+v"(r[j]));
#pragma unroll
            for (int f = 0; f < NF; ++f)
                asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[j]) : "v"(b), "v"(c));
        }
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j] + r[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst,
                       size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

}  // namespace

// kind: 0 fma, 1 exp, 2 rcp, 10+nf mix (1 rcp + nf fma).  Returns the
// kernel time in ms (best of `reps`) for blocks x threads lanes, or < 0.
UB_API double xrdvi_ubench_alu(int kind, int blocks, int threads, int iters,
                               int reps) {
    if (blocks < 1 || threads < 64 || threads > 1024 || (threads % 64) ||
        iters < 1 || reps < 1)
        return -1.0;
    float *out = nullptr;
    if (hipMalloc(&out, sizeof(float) * (size_t)blocks * threads) != hipSuccess)
        return -2.0;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, nullptr);
        switch (kind) {
            case 0: k_fma<<<blocks, threads>>>(out, iters, 0.999f, 1e-3f); break;
            case 1: k_exp<<<blocks, threads>>>(out, iters); break;
            case 2: k_rcp<<<blocks, threads>>>(out, iters); break;
            case 11: k_mix<1><<<blocks, threads>>>(out, iters, 0.999f, 1e-3f); break;
            case 12: k_mix<2><<<blocks, threads>>>(out, iters, 0.999f, 1e-3f); break;
            case 14: k_mix<4><<<blocks, threads>>>(out, iters, 0.999f, 1e-3f); break;
            default: (void)hipFree(out); return -1.0;
        }
        (void)hipEventRecord(e1, nullptr);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return hipGetLastError() == hipSuccess ? best : -3.0;
}

// Copies `bytes` (multiple of 16) device-to-device with a plain kernel;
// returns the best time in ms.
UB_API double xrdvi_ubench_copy(size_t bytes, int reps) {
    if (bytes < 16 || bytes % 16 || reps < 1) return -1.0;
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return -2.0;
    if (hipMalloc(&b, bytes) != hipSuccess) { (void)hipFree(a); return -2.0; }
    (void)hipMemset(a, 0, bytes);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    double best = 1e30;
    const size_t n = bytes / 16;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, nullptr);
        k_copy<<<4096, 256>>>((const float4 *)a, (float4 *)b, n);
        (void)hipEventRecord(e1, nullptr);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    return hipGetLastError() == hipSuccess ? best : -3.0;
}
