// Attainable issue rates of the units the blend kernels use, measured on the device: FP32 FMA
// (not packed), the transcendental exp2, and the FP16 MFMA of the exponent product. Each kernel
// runs independent dependency chains in every lane so that issue, not latency, bounds it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;

__global__ __launch_bounds__(256) void k_fma(float *out, int iters, float b, float c) {
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = float(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = fmaf(a[k], b, c);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_exp(float *out, int iters, float b) {
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = -float(threadIdx.x & 7) - 0.125f * k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = __builtin_amdgcn_exp2f(a[k]) * b;
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_mfma(float *out, int iters) {
    h8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) { a[k] = _Float16(0.001f * (threadIdx.x + k)); b[k] = _Float16(0.5f); }
    f16x acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[c][k] = 0.f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int k = 0; k < 16; ++k) s += acc[c][k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// which: 0 = FMA, 1 = exp2, 2 = MFMA 32x32x16 f16. blocks x 256 threads, `iters` iterations of
// the inner step. Returns the kernel time in ms (HIP events, after one warm-up launch) and the
// operation count: FMAs, exp2s, or MFMA instructions (per wavefront) issued in total.
extern "C" int gsbpk_run(int which, int blocks, int iters, float *ms, double *ops) {
    float *buf = nullptr;
    if (hipMalloc(&buf, sizeof(float) * size_t(blocks) * 256) != hipSuccess) return 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, nullptr);
        if (which == 0) k_fma<<<blocks, 256>>>(buf, iters, 0.999f, 0.001f);
        else if (which == 1) k_exp<<<blocks, 256>>>(buf, iters, 0.5f);
        else k_mfma<<<blocks, 256>>>(buf, iters);
        if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    }
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    const double threads = double(blocks) * 256.0;
    if (which == 0) *ops = threads * iters * kChains;
    else if (which == 1) *ops = threads * iters * kChains;
    else *ops = threads / 64.0 * iters * 4;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    const hipError_t err = hipGetLastError();
    (void)hipFree(buf);
    return e == hipSuccess && err == hipSuccess ? 0 : 2;
}
