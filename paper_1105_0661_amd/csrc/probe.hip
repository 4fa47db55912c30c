// probe.hip -- peak probes for roofline reporting: register-only MFMA loops
// (the instruction forms the contraction uses), a plain device copy and a
// read-only stream.
// They measure what this device sustains, beside the datasheet figures.
#include "lbf_device.h"
#include "lbf_launch.h"

namespace lbf {

typedef _Float16 halfx8p __attribute__((ext_vector_type(8)));

// 4-wave work groups, 2 per compute unit (two waves per SIMD, as the fast
// workers), 8 independent accumulator chains
// per wave (each MFMA depends on the previous one of its chain, so the loop
// cannot be folded).
__global__ __launch_bounds__(256) void probe_mfma_f16_kernel(float* sink, int iters) {
    halfx8p a, b;
    for (int i = 0; i < 8; ++i) {
        a[i] = (_Float16)(0.001f * (float)((threadIdx.x * 7 + i) & 255));
        b[i] = (_Float16)(0.002f * (float)((threadIdx.x * 3 + i) & 127));
    }
    floatx16 acc[8];
    for (int j = 0; j < 8; ++j) acc[j] = floatx16{};
    __asm__ volatile("" : "+v"(a), "+v"(b));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.f;
    for (int j = 0; j < 8; ++j) s += acc[j][j];
    if (s == 1234.5f) sink[threadIdx.x] = s;   // never true; keeps the chains live
}

__global__ __launch_bounds__(256) void probe_mfma_f32_kernel(float* sink, int iters) {
    float a = 0.001f * (float)(threadIdx.x & 255), b = 0.002f * (float)((threadIdx.x * 5) & 127);
    floatx16 acc[8];
    for (int j = 0; j < 8; ++j) acc[j] = floatx16{};
    __asm__ volatile("" : "+v"(a), "+v"(b));
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.f;
    for (int j = 0; j < 8; ++j) s += acc[j][j];
    if (s == 1234.5f) sink[threadIdx.x] = s;
}

// 16-byte copy, four elements per thread in flight; n4 = number of 16-byte
// elements
__global__ __launch_bounds__(256) void probe_copy_kernel(const floatx4* __restrict__ src, floatx4* __restrict__ dst,
                                                         size_t n4) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += 4 * stride) {
        floatx4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * stride < n4) v[u] = __builtin_nontemporal_load(src + i + u * stride);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i + u * stride < n4) __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
}

// 16-byte read stream, four loads per thread in flight, folded into an xor
// that is stored only where it equals `key` (so the loads stay live; dst
// takes at most one word per thread index, 256 words)
__global__ __launch_bounds__(256) void probe_read_kernel(const floatx4* __restrict__ src, uint32_t* __restrict__ dst,
                                                         size_t n4, uint32_t key) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += 4 * stride) {
        floatx4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            v[u] = floatx4{};
            if (i + u * stride < n4) v[u] = __builtin_nontemporal_load(src + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc ^= __float_as_uint(v[u][0]) ^ __float_as_uint(v[u][1]) ^ __float_as_uint(v[u][2]) ^
                   __float_as_uint(v[u][3]);
    }
    if (acc == key) dst[threadIdx.x] = acc;
}

hipError_t launch_probe(int kind, int iters, const void* src, void* dst, size_t bytes, double* work, hipStream_t st) {
    int dev = 0, cus = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (kind == 0 || kind == 1) {
        // two 256-thread work groups per compute unit; `dst` receives
        // nothing unless the impossible sink condition holds (it never does)
        const int grid = 2 * cus;
        if (kind == 0) hipLaunchKernelGGL(probe_mfma_f16_kernel, dim3(grid), dim3(256), 0, st, (float*)dst, iters);
        else hipLaunchKernelGGL(probe_mfma_f32_kernel, dim3(grid), dim3(256), 0, st, (float*)dst, iters);
        *work = (double)grid * 4 * (double)iters * 8 * (kind == 0 ? 32768.0 : 4096.0);
        return hipGetLastError();
    }
    const size_t n4 = bytes / 16;
    if (kind == 3) {
        hipLaunchKernelGGL(probe_read_kernel, dim3((unsigned)(cus * 32)), dim3(256), 0, st, (const floatx4*)src,
                           (uint32_t*)dst, n4, 0x9e3779b9u);
        *work = (double)(n4 * 16);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(probe_copy_kernel, dim3((unsigned)(cus * 32)), dim3(256), 0, st, (const floatx4*)src,
                       (floatx4*)dst, n4);
    *work = 2.0 * (double)(n4 * 16);
    return hipGetLastError();
}

}  // namespace lbf
