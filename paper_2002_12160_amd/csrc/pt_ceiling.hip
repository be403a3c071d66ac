// pt_ceiling.hip -- microbenchmarks of the two ceilings the hot path's
// kernels are measured against, on the device they run on: the float64 FMA
// rate of the vector ALUs and the HBM copy bandwidth.  Built as its own
// library (libptceil.so); the hot path does not use it.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

constexpr int CHAINS = 8;

// every thread runs CHAINS independent FMA chains for `iters` rounds
// (x <- x a + b converges to b / (1 - a), so the values stay normal)
__global__ void __launch_bounds__(256) k_fma_f64(double *out, int iters, double a, double b)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    double x[CHAINS];
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) x[c] = 1.0 + 1e-3 * c + 1e-9 * gid;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < CHAINS; ++c) x[c] = __fma_rn(x[c], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CHAINS; ++c) s += x[c];
    out[gid] = s;
}

// grid-stride copy of n 16-byte words
__global__ void __launch_bounds__(256) k_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// FMA loop on blocks x 256 threads; out: device, blocks * 256 doubles.
// Floating-point operations done: 2 * CHAINS * iters * blocks * 256.
// Returns a hipError_t value (0 on success).
__attribute__((visibility("default"))) int ptc_fma_f64(double *out, int blocks, int iters, void *stream)
{
    if (!out || blocks < 1 || iters < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fma_f64, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters, 0.999999, 1e-6);
    return (int)hipGetLastError();
}

__attribute__((visibility("default"))) int ptc_fma_chains(void) { return CHAINS; }

// Copy of `bytes` (a multiple of 16; both pointers 16-byte aligned device
// memory) on `blocks` x 256 threads.  Returns a hipError_t value.
__attribute__((visibility("default"))) int ptc_copy(const void *src, void *dst, size_t bytes, int blocks, void *stream)
{
    if (!src || !dst || bytes % 16 != 0 || blocks < 1 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
        return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (const float4 *)src, (float4 *)dst,
                       bytes / 16);
    return (int)hipGetLastError();
}

}  // extern "C"
