// Calibration kernels: a plain vectorised copy, streaming read / write / copy
// probes for the HBM ceilings, and an FMA-throughput loop.
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

// Streaming probes for the HBM ceilings: each thread moves 4 x 16 bytes per
// step (four independent accesses a grid stride apart, all in flight at
// once), with plain or non-temporal stores.
typedef int v4i __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ void put(v4i* p, v4i v)
{
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// read only: an XOR of everything read, one 16-byte word per workgroup out
__global__ __launch_bounds__(256) void k_sread(const v4i* __restrict__ src, int64_t n, v4i* __restrict__ sink)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    v4i acc = {0, 0, 0, 0};
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4i a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        acc ^= a ^ b ^ c ^ d;
    }
    for (; i < n; i += stride)
        acc ^= src[i];
    __shared__ int red[256];
    red[threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int k = 0; k < 256; ++k)
            r ^= red[k];
        sink[blockIdx.x] = v4i{r, 0, 0, 0};
    }
}

template <bool NT>
__global__ __launch_bounds__(256) void k_swrite(v4i* __restrict__ dst, int64_t n, int value)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    const v4i v = {value, value + 1, value + 2, value + 3};
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        put<NT>(dst + i, v);
        put<NT>(dst + i + stride, v);
        put<NT>(dst + i + 2 * stride, v);
        put<NT>(dst + i + 3 * stride, v);
    }
    for (; i < n; i += stride)
        put<NT>(dst + i, v);
}

template <bool NT>
__global__ __launch_bounds__(256) void k_scopy(v4i* __restrict__ dst, const v4i* __restrict__ src, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4i a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        put<NT>(dst + i, a);
        put<NT>(dst + i + stride, b);
        put<NT>(dst + i + 2 * stride, c);
        put<NT>(dst + i + 3 * stride, d);
    }
    for (; i < n; i += stride)
        put<NT>(dst + i, src[i]);
}

// Chunked write: 8 KiB chunks, each written by one workgroup as a lane's two
// 16-byte stores 32 bytes apart (the store pattern of a tile of 1024 cf32
// outputs at four per lane).  Chunk q belongs to stream q mod S at position
// q div S, the streams being S equal slices of the buffer, so S sets how
// many separate regions the running workgroups write at once.
template <bool NT>
__global__ __launch_bounds__(256) void k_schunk(v4i* __restrict__ dst, int64_t chunks, int64_t streams)
{
    const int64_t per_stream = chunks / streams;
    const v4i v = {1, 2, 3, 4};
    for (int64_t q = blockIdx.x; q < per_stream * streams; q += gridDim.x) {
        const int64_t s = q % streams, j = q / streams;
        v4i* c = dst + (s * per_stream + j) * 512;  // 512 x 16 bytes per chunk
        put<NT>(c + 2 * threadIdx.x, v);
        put<NT>(c + 2 * threadIdx.x + 1, v);
    }
}

}  // namespace

extern "C" int32_t tt_probe_chunked_write(void* dst, int64_t bytes, int32_t streams, int32_t blocks,
                                          int32_t nontemporal, void* hip_stream)
{
    const int64_t chunks = bytes / 8192;
    if (!dst || bytes % 8192 || streams < 1 || chunks < streams || blocks < 1 || blocks > (1 << 20))
        return (int32_t)hipErrorInvalidValue;
    if (nontemporal)
        hipLaunchKernelGGL(k_schunk<true>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                           (v4i*)dst, chunks, (int64_t)streams);
    else
        hipLaunchKernelGGL(k_schunk<false>, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                           (v4i*)dst, chunks, (int64_t)streams);
    return (int32_t)hipGetLastError();
}

extern "C" int32_t tt_probe_stream(int32_t kind, void* dst, const void* src, int64_t bytes, int32_t blocks,
                                   int32_t nontemporal, void* hip_stream)
{
    if (bytes < 16 || bytes % 16 || blocks < 1 || blocks > (1 << 20) || kind < 0 || kind > 2)
        return (int32_t)hipErrorInvalidValue;
    if ((kind != 1 && !src) || !dst)
        return (int32_t)hipErrorInvalidValue;
    const int64_t n = bytes / 16;
    hipStream_t st = (hipStream_t)hip_stream;
    if (kind == 0)
        hipLaunchKernelGGL(k_sread, dim3((unsigned)blocks), dim3(256), 0, st, (const v4i*)src, n, (v4i*)dst);
    else if (kind == 1 && nontemporal)
        hipLaunchKernelGGL(k_swrite<true>, dim3((unsigned)blocks), dim3(256), 0, st, (v4i*)dst, n, 7);
    else if (kind == 1)
        hipLaunchKernelGGL(k_swrite<false>, dim3((unsigned)blocks), dim3(256), 0, st, (v4i*)dst, n, 7);
    else if (nontemporal)
        hipLaunchKernelGGL(k_scopy<true>, dim3((unsigned)blocks), dim3(256), 0, st, (v4i*)dst, (const v4i*)src, n);
    else
        hipLaunchKernelGGL(k_scopy<false>, dim3((unsigned)blocks), dim3(256), 0, st, (v4i*)dst, (const v4i*)src, n);
    return (int32_t)hipGetLastError();
}

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
