// gfx950 kernel for trace replay from continuous-delay CIRs (Sec. IV, channel
// traces: complex taps uniformly spaced in delay, one snapshot per time step).
//
// k_resample: one workgroup of four wave64 per (entry, time step); lane l of
// every wave works on grid tap l (L <= 64) for every antenna pair of the step,
//   H_k[r][t][l] = sum_p a_{k,p,r,t} sinc(fs (tau_{k,p} - t0) - l),
// with sinc(x) = sin(pi x) / (pi x), in FP64: each wave sums a contiguous
// quarter of the paths in index order, the quarters are added in order, and
// the sum is rounded once to the ring's storage format into ring slot
// (k0 + step) mod cap.  The work per step is n_paths * (one sinc + n_rx n_tx
// complex products) per lane, small beside the convolution the snapshot then
// feeds; FP64 keeps the rounding to the one final conversion.
#include "tt_internal.h"

namespace tt {

namespace {

constexpr int kMaxPairs = kMaxAnt * kMaxAnt;

__device__ inline double sinc_pi(double x)
{
    return x == 0.0 ? 1.0 : sinpi(x) / (M_PI * x);
}

}  // namespace

// grid: (entries, steps clamped to 65535), block: kResWaves wave64.  Wave w
// sums the w-th contiguous quarter of the paths; wave 0 then adds the other
// quarters in wave order, so the result does not depend on timing.
constexpr int kResWaves = 4;

__global__ __launch_bounds__(64 * kResWaves) void k_resample(const ResampleDev* __restrict__ ent)
{
    __shared__ double2 part[kResWaves - 1][kMaxPairs][64];
    const ResampleDev& e = ent[blockIdx.x];
    const int l = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int nrt = e.n_rx * e.n_tx;
    const int64_t per = (int64_t)nrt * e.L;
    const int chunk = (e.n_paths + kResWaves - 1) / kResWaves;
    const int p0 = min(e.n_paths, wv * chunk), p1 = min(e.n_paths, p0 + chunk);
    for (int s = blockIdx.y; s < e.count; s += gridDim.y) {
        double2 acc[kMaxPairs];
#pragma unroll
        for (int q = 0; q < kMaxPairs; ++q)
            acc[q] = make_double2(0.0, 0.0);
        const double* dl = e.delay + (int64_t)s * e.n_paths;
        const float2* g = e.gain + (int64_t)s * e.n_paths * nrt;
        for (int p = p0; p < p1; ++p) {
            const double k = sinc_pi((dl[p] - e.t0) * e.fs - (double)l);
#pragma unroll
            for (int q = 0; q < kMaxPairs; ++q) {
                if (q < nrt) {
                    const float2 a = g[(int64_t)p * nrt + q];
                    acc[q].x += (double)a.x * k;
                    acc[q].y += (double)a.y * k;
                }
            }
        }
        if (wv > 0) {
#pragma unroll
            for (int q = 0; q < kMaxPairs; ++q)
                if (q < nrt)
                    part[wv - 1][q][l] = acc[q];
        }
        __syncthreads();
        if (wv == 0 && l < e.L) {
            const int64_t base = ((e.k0 + s) % e.cap) * per + l;
#pragma unroll
            for (int q = 0; q < kMaxPairs; ++q) {
                if (q < nrt) {
                    double2 v = acc[q];
#pragma unroll
                    for (int w = 0; w < kResWaves - 1; ++w) {
                        v.x += part[w][q][l].x;
                        v.y += part[w][q][l].y;
                    }
                    if (e.tap_fmt == TAP_F16) {
                        // one correctly rounded FP64 -> FP16 conversion per component
                        const _Float16 hx = (_Float16)v.x, hy = (_Float16)v.y;
                        uint16_t bx, by;
                        __builtin_memcpy(&bx, &hx, 2);
                        __builtin_memcpy(&by, &hy, 2);
                        reinterpret_cast<uint32_t*>(e.ring)[base + (int64_t)q * e.L] = ((uint32_t)by << 16) | bx;
                    } else {
                        reinterpret_cast<float2*>(e.ring)[base + (int64_t)q * e.L] =
                            make_float2((float)v.x, (float)v.y);
                    }
                }
            }
        }
        // the partials are read before the next step overwrites them
        __syncthreads();
    }
}

hipError_t launch_resample(const ResampleDev* ent, int n, int max_count, hipStream_t st)
{
    if (n <= 0 || max_count <= 0)
        return hipSuccess;
    const unsigned steps = (unsigned)(max_count < 65535 ? max_count : 65535);
    hipLaunchKernelGGL(k_resample, dim3((unsigned)n, steps), dim3(64 * kResWaves), 0, st, ent);
    return hipGetLastError();
}

}  // namespace tt
