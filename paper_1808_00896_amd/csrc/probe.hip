// probe.hip -- the device ceilings the roofline fractions are read against,
// measured with kernels of this library rather than a vendor library: a
// streaming copy (the HBM rate a pass that reads and writes every byte once
// can reach) and dependent-chain loops on the FP64 vector unit and on the
// FP64 and FP32 matrix cores (the rates the DWT contractions can reach).
#include "soft_internal.h"

namespace soft {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

// Copy of n 16-byte words, four per thread and iteration (all loads issued
// before any store), with non-temporal loads and stores: every byte is read
// once and written once.
__global__ __launch_bounds__(256) void k_probe_copy(const u4 *__restrict__ src, u4 *__restrict__ dst, long long n) {
    const long long stride = (long long)gridDim.x * 256 * 4;
    long long i = (long long)blockIdx.x * 256 * 4 + threadIdx.x;
    for (; i + 3 * 256 < n; i += stride) {
        u4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load(src + i + u * 256);
#pragma unroll
        for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * 256);
    }
    for (; i < n; i += 256) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// FP64 vector FMA loop: eight independent chains per lane, `iters` rounds.
__global__ __launch_bounds__(256) void k_probe_fma64(int iters, double *__restrict__ sink) {
    const double b = 1.0 + 1e-12 * threadIdx.x, c = 1e-9;
    double a[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = (double)(q + 1) + threadIdx.x;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = fma(a[q], b, c);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += a[q];
    if (s == 1.2345) sink[blockIdx.x * 256 + threadIdx.x] = s;  // keeps the chains live
}

// FP64 matrix-core loop: v_mfma_f64_16x16x4, four independent accumulator
// chains, two rounds of them per iteration (8 MFMAs).
__global__ __launch_bounds__(256) void k_probe_mfma64(int iters, double *__restrict__ sink) {
    const double a = 1.0 + 1e-12 * threadIdx.x, b = 1.0 - 1e-12 * threadIdx.x;
    v4d acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (v4d){0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r & 3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[r & 3], 0, 0, 0);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    if (s == 1.2345) sink[blockIdx.x * 256 + threadIdx.x] = s;
}

// FP32 matrix-core loop: v_mfma_f32_16x16x4f32 (the instruction of the FP32
// DWT contractions), as above.
__global__ __launch_bounds__(256) void k_probe_mfma32(int iters, double *__restrict__ sink) {
    const float a = 1.0f + 1e-6f * threadIdx.x, b = 1.0f - 1e-6f * threadIdx.x;
    v4f acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (v4f){0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r & 3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[r & 3], 0, 0, 0);
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    if (s == 1.2345f) sink[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_probe_copy(const void *src, void *dst, long long words, hipStream_t s) {
    long long blocks = (words + 1023) / 1024;
    if (blocks > 256 * 32) blocks = 256 * 32;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_probe_copy, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const u4 *>(src),
                       static_cast<u4 *>(dst), words);
    return hipGetLastError();
}

hipError_t launch_probe_flops(int kind, int blocks, int iters, double *sink, hipStream_t s) {
    switch (kind) {
        case 0: hipLaunchKernelGGL(k_probe_fma64, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        case 1: hipLaunchKernelGGL(k_probe_mfma64, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        case 2: hipLaunchKernelGGL(k_probe_mfma32, dim3(blocks), dim3(256), 0, s, iters, sink); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Flops of one launch: per wave and iteration, 8 FMAs on 64 lanes (FMA =
// 2 flops) for the vector loop, 8 MFMAs of 16x16x4 (2 * 16 * 16 * 4 flops)
// for the matrix loops; 4 waves per block.
double probe_flop_count(int kind, int blocks, int iters) {
    const double per_wave_iter = kind == 0 ? 8.0 * 64 * 2 : 8.0 * 2 * 16 * 16 * 4;
    return per_wave_iter * 4.0 * (double)blocks * (double)iters;
}

}  // namespace soft
