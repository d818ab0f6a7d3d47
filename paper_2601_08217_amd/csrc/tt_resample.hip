// gfx950 kernel for trace replay from continuous-delay CIRs (Sec. IV, channel
// traces: complex taps uniformly spaced in delay, one snapshot per time step).
//
// k_resample: one wave64 per (entry, time step); lane l computes grid tap l
// (L <= 64) for every antenna pair of the step,
//   H_k[r][t][l] = sum_p a_{k,p,r,t} sinc(fs (tau_{k,p} - t0) - l),
// with sinc(x) = sin(pi x) / (pi x), in FP64 with paths summed in index order,
// then rounds once to the ring's storage format and writes ring slot
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

// grid: (entries, steps clamped to 65535), block: one wave64
__global__ __launch_bounds__(64) void k_resample(const ResampleDev* __restrict__ ent)
{
    const ResampleDev& e = ent[blockIdx.x];
    const int l = threadIdx.x;
    const int nrt = e.n_rx * e.n_tx;
    const int64_t per = (int64_t)nrt * e.L;
    for (int s = blockIdx.y; s < e.count; s += gridDim.y) {
        double2 acc[kMaxPairs];
#pragma unroll
        for (int q = 0; q < kMaxPairs; ++q)
            acc[q] = make_double2(0.0, 0.0);
        const double* dl = e.delay + (int64_t)s * e.n_paths;
        const float2* g = e.gain + (int64_t)s * e.n_paths * nrt;
        for (int p = 0; p < e.n_paths; ++p) {
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
        if (l < e.L) {
            const int64_t base = ((e.k0 + s) % e.cap) * per + l;
#pragma unroll
            for (int q = 0; q < kMaxPairs; ++q) {
                if (q < nrt) {
                    if (e.tap_fmt == TAP_F16) {
                        // one correctly rounded FP64 -> FP16 conversion per component
                        const _Float16 hx = (_Float16)acc[q].x, hy = (_Float16)acc[q].y;
                        uint16_t bx, by;
                        __builtin_memcpy(&bx, &hx, 2);
                        __builtin_memcpy(&by, &hy, 2);
                        reinterpret_cast<uint32_t*>(e.ring)[base + (int64_t)q * e.L] = ((uint32_t)by << 16) | bx;
                    } else {
                        reinterpret_cast<float2*>(e.ring)[base + (int64_t)q * e.L] =
                            make_float2((float)acc[q].x, (float)acc[q].y);
                    }
                }
            }
        }
    }
}

hipError_t launch_resample(const ResampleDev* ent, int n, int max_count, hipStream_t st)
{
    if (n <= 0 || max_count <= 0)
        return hipSuccess;
    const unsigned steps = (unsigned)(max_count < 65535 ? max_count : 65535);
    hipLaunchKernelGGL(k_resample, dim3((unsigned)n, steps), dim3(64), 0, st, ent);
    return hipGetLastError();
}

}  // namespace tt
