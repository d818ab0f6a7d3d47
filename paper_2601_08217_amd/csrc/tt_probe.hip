// Calibration kernels: a plain vectorised copy and an FMA-throughput loop.
#include <hip/hip_runtime.h>

#include "tt_probe.h"

namespace {

__global__ __launch_bounds__(256) void k_copy(int4* __restrict__ dst, const int4* __restrict__ src, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_fma(float* __restrict__ out, int iters)
{
    float a[16];
    const float m = 1.0f + 1e-7f * (float)threadIdx.x, c = 1e-7f;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        a[j] = (float)(threadIdx.x + j);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int j = 0; j < 16; ++j)
                a[j] = fmaf(a[j], m, c);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 16; ++j)
        s += a[j];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

extern "C" int32_t tt_probe_copy(void* dst, const void* src, int64_t bytes, void* hip_stream)
{
    if (!dst || !src || bytes < 0 || bytes % 16)
        return (int32_t)hipErrorInvalidValue;
    const int64_t n = bytes / 16;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64)
        blocks = 256 * 64;
    if (blocks < 1)
        return 0;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream, (int4*)dst,
                       (const int4*)src, n);
    return (int32_t)hipGetLastError();
}

extern "C" int32_t tt_probe_fma(float* out, int32_t blocks, int32_t iters, void* hip_stream)
{
    if (!out || blocks < 1 || iters < 1)
        return (int32_t)hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fma, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, out, iters);
    return (int32_t)hipGetLastError();
}
