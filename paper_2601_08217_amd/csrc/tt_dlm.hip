// gfx950 matrix-core path of the broadcast downlink.
//
// The gNB transmits one raw stream that every UE of the cell convolves with
// its own channel (Tiny-Twin, Sec. III-B, the rfsim paragraph), so over one
// snapshot block the downlink of a group of UEs is a dense contraction:
//
//   Y[u, r][n] = sum_{t, l} T[u, r, t, l] x_t[n - l],   T = H_k or D_k,
//
// (UEs x taps) times a Hankel matrix of the shared input (taps x time).  With
// h = H + a D (a = offset of n inside the block) the output is
// y = Y_H + a Y_D.  The contraction runs on f16 MFMA
// (v_mfma_f32_32x32x16_f16, FP32 accumulation) with exact operand splits:
//   - the ci16 input x = x_hi + x_lo, x_hi the multiple of 32 below x and
//     x_lo in [0, 32): both are exact in f16;
//   - the taps, scaled per (UE, rx) by a power of two so that the largest
//     component lies in [2^14, 2^15), T' = T_hi + T_lo with T_hi the f16
//     rounding of T' and T_lo the f16 rounding of T' - T_hi (22 significant
//     bits together).
// All four cross products are accumulated, so each product term carries a
// relative error of a few 2^-22 before the FP32 sum; the power-of-two scale
// is undone exactly in the epilogue.
//
// One workgroup (4 wave64) covers 16 (UE, rx) rows of one DL group over
// kDlmBlocks blocks of 128 samples.  Wave w owns rows 4w .. 4w + 3 (one
// 32-row matrix tile) and all four 32-sample column tiles of each block: it
// stages its rows' taps, builds its A operand table in LDS, prefetches the
// next block's snapshot and runs 4 x KS MFMAs per block (one A read per four
// MFMAs); the input tile is staged once for all waves.  Matrix layout of one wave and block:
//   rows    (32): (UE, rx) row u in 0..3, tap split part s_h, and
//                 c = 2 * (H or D) + complex output part;
//                 row i: u = 2 (i / 16) + (i / 4) % 2, s_h = (i / 8) % 2,
//                 c = i % 4, which puts the eight values of one (u, n) in
//                 one lane of the MFMA result;
//   depth   (16 per instruction): two consecutive taps of one transmit
//                 stream per half wave, x complex input part x split part;
//   columns (4 x 32): output samples of the block.
// The UEs' own histories are not part of the shared input: in the call's
// first block the input before the call is zero in the product, and each
// output n < L - 1 adds its history terms in FP32 afterwards.
#include "tt_internal.h"

namespace tt {

extern __shared__ __align__(16) unsigned char g_lds_m[];

namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float float16v __attribute__((ext_vector_type(16)));

// ci16 sample (int16 counts) -> (re_hi, re_lo, im_hi, im_lo)
__device__ __forceinline__ uint2 split_x(uint32_t w)
{
    const int re = (int16_t)(w & 0xffffu), im = (int32_t)w >> 16;
    const int rh = re & ~31, ih = im & ~31;
    const _Float16 v[4] = {(_Float16)rh, (_Float16)(re - rh), (_Float16)ih, (_Float16)(im - ih)};
    uint2 o;
    __builtin_memcpy(&o, v, 8);
    return o;
}

__device__ __forceinline__ uint32_t encode(float a, float b, int* sat)
{
    float x = rintf(a), y = rintf(b);
    *sat += (x > 32767.0f || x < -32768.0f) + (y > 32767.0f || y < -32768.0f);
    x = fminf(fmaxf(x, -32768.0f), 32767.0f);
    y = fminf(fmaxf(y, -32768.0f), 32767.0f);
    return (uint32_t)(uint16_t)(int16_t)x | ((uint32_t)(uint16_t)(int16_t)y << 16);
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_dlm(const JobDev* __restrict__ jobs, int njobs, int tiles_per_job,
                                                const LinkDev* __restrict__ links,
                                                const __half2* __restrict__ noise, int32_t npool,
                                                unsigned long long* __restrict__ sat)
{
    constexpr int TM = kDlmBlocks * 128;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, j = lane & 31;
    const int tile = blockIdx.x;
    int ji;
    if (tiles_per_job > 0) {
        ji = tile / tiles_per_job;
    } else {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].tile0 <= tile)
                lo = mid;
            else
                hi = mid - 1;
        }
        ji = lo;
    }
    const JobDev& job = jobs[ji];
    const LinkDev& l0 = links[job.link0];
    const int N = job.N;
    const int i0 = (tile - job.tile0) * TM;
    const int n_tx = l0.n_tx, n_rx = l0.n_rx, L = l0.L, P = l0.period;
    const bool linear = l0.mode == M_LINEAR;
    const int nu = job.nlinks * n_rx;  // (UE, rx) rows in use, <= 16
    const int Lq = (L + 1) & ~1;
    const int TL = n_tx * Lq;            // (tx, tap) entries per row
    const int KS = (TL + 3) / 4;         // MFMA depth steps (<= 8)
    const int XS = TM + Lq;
    uint2* xs = reinterpret_cast<uint2*>(g_lds_m);
    float4* tw = reinterpret_cast<float4*>(g_lds_m + ((n_tx * XS * 8 + 15) & ~15)) + wave * 4 * TL;
    uint4* aw = reinterpret_cast<uint4*>(g_lds_m + ((n_tx * XS * 8 + 15) & ~15) + 4 * 4 * TL * 16) + wave * KS * 64;
    __shared__ int s_mx[16];
    int nsat = 0;

    // shared input of the tile (plus the taps' reach before it); samples
    // before the call or past its end are zero
    const int s0 = i0 - Lq;
    const uint32_t* xg = reinterpret_cast<const uint32_t*>(l0.x);
    for (int e = tid; e < n_tx * XS; e += kBlock) {
        const int t = e / XS;
        const int p = e - t * XS;
        const int s = s0 + p;
        xs[e] = (s >= 0 && s < N) ? split_x(xg[(int64_t)t * N + s]) : make_uint2(0u, 0u);
    }

    // this lane's tap entries: row u = lane / 16 of the wave's rows, entries
    // q = lane % 16 + 16 m (m < 2) of that row's (tx, tap) list
    const int u_me = lane >> 4;
    const int row_me = 4 * wave + u_me;
    const bool row_ok = row_me < nu;
    const LinkDev& lk_me = links[job.link0 + (row_ok ? row_me / n_rx : 0)];
    const int r_me = row_ok ? row_me % n_rx : 0;
    int off_me[2];
    bool ok_me[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int q = (lane & 15) + 16 * m;
        const int t = q / Lq;
        const int l = q - t * Lq;
        ok_me[m] = row_ok && q < TL && l < L;
        off_me[m] = (r_me * n_tx + t) * L + l;
    }
    auto load = [&](int64_t koff_q, float2 (&v)[2]) {
        const int64_t k = lk_me.k0 + koff_q;
        const int64_t slot = lk_me.ring_cap ? k % lk_me.ring_cap : k - lk_me.kbase;
        const int64_t base = slot * (lk_me.n_rx * lk_me.n_tx * lk_me.L);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            v[m] = make_float2(0.f, 0.f);
            if (ok_me[m]) {
                const int64_t idx = base + off_me[m];
                v[m] = lk_me.tap_fmt == TAP_F16 ? __half22float2(reinterpret_cast<const __half2*>(lk_me.ring)[idx])
                                                : reinterpret_cast<const float2*>(lk_me.ring)[idx];
            }
        }
    };
    float2 sa[2], sb[2], pf[2];
    int64_t have = -1, pf_k = -1;
    float unscale[2] = {1.f, 1.f};

    for (int b = 0; b < kDlmBlocks; ++b) {
        const int nb0 = b * 128;
        if (i0 + nb0 >= N)
            break;
        const int64_t koff = (i0 + nb0) / P;
        if (koff != have) {
            // snapshots koff (and koff + 1 for LINEAR) of the lane's entries
            const bool next = have >= 0 && koff == have + 1;
            if (linear) {
                if (next) {
                    sa[0] = sb[0];
                    sa[1] = sb[1];
                } else {
                    load(koff, sa);
                }
                if (pf_k == koff + 1) {
                    sb[0] = pf[0];
                    sb[1] = pf[1];
                } else {
                    load(koff + 1, sb);
                }
            } else if (pf_k == koff) {
                sa[0] = pf[0];
                sa[1] = pf[1];
            } else {
                load(koff, sa);
            }
            have = koff;
            __syncthreads();  // the previous block's taps and maxima are no longer read
            if (tid < 16)
                s_mx[tid] = 0;
            __syncthreads();
            const float inv_p = 1.0f / (float)P;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int q = (lane & 15) + 16 * m;
                if (q < TL) {
                    float4 v = make_float4(sa[m].x, sa[m].y, 0.f, 0.f);
                    if (linear) {
                        v.z = (sb[m].x - sa[m].x) * inv_p;
                        v.w = (sb[m].y - sa[m].y) * inv_p;
                    }
                    tw[u_me * TL + q] = v;
                    const float mx = fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w)));
                    atomicMax(&s_mx[row_me & 15], __float_as_int(mx));
                }
            }
            __syncthreads();
            // per-row power-of-two scales: largest component in [2^14, 2^15)
            auto row_scale = [&](int row, float* sc, float* usc) {
                const float m = __int_as_float(s_mx[row]);
                int ex = 0;
                if (m > 0.f)
                    (void)frexpf(m, &ex);
                const int sh = m > 0.f ? min(15 - ex, 126) : 0;
                *sc = ldexpf(1.0f, sh);
                *usc = ldexpf(1.0f, -sh);
            };
            {
                float tmp;
                row_scale(4 * wave + h, &tmp, &unscale[0]);
                row_scale(4 * wave + 2 + h, &tmp, &unscale[1]);
            }
            // A operand table of the wave: entry (kk, lane) = row i = j, half h
            {
                const int i = j;
                const int u = 2 * (i >> 4) + ((i >> 2) & 1);
                const int sh = (i >> 3) & 1;
                const int c = i & 3;
                const int hd = c >> 1, cout = c & 1;
                float srow, tmp;
                row_scale(4 * wave + u, &srow, &tmp);
                for (int kk = 0; kk < KS; ++kk) {
                    const int p0 = 4 * kk + 2 * h;  // (t, l) pair: taps l0 + 1 then l0
                    _Float16 v8[8];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const int p = p0 + 1 - q;
                        const int t = p / Lq;
                        const int l = p - t * Lq;
                        float re = 0.f, im = 0.f;
                        if (t < n_tx) {
                            const float4 v = tw[u * TL + t * Lq + l];
                            re = (hd ? v.z : v.x) * srow;
                            im = (hd ? v.w : v.y) * srow;
                        }
                        // output part from (input re, input im): re <- (re, -im), im <- (im, re)
                        const float f_re = cout ? im : re;
                        const float f_im = cout ? re : -im;
#pragma unroll
                        for (int cin = 0; cin < 2; ++cin) {
                            const float f = cin ? f_im : f_re;
                            const _Float16 fh = (_Float16)f;
                            const _Float16 part = sh ? (_Float16)(f - (float)fh) : fh;
                            v8[4 * q + 2 * cin + 0] = part;  // input split hi
                            v8[4 * q + 2 * cin + 1] = part;  // input split lo
                        }
                    }
                    uint4 o;
                    __builtin_memcpy(&o, v8, 16);
                    aw[kk * 64 + lane] = o;
                }
            }
            __syncthreads();
        }
        // prefetch the snapshot the next block adds
        if (b + 1 < kDlmBlocks && i0 + nb0 + 128 < N) {
            const int64_t kn = (i0 + nb0 + 128) / P;
            if (kn != koff) {
                pf_k = linear ? kn + 1 : kn;
                load(pf_k, pf);
            }
        }

        // contraction: four column tiles of 32 samples
        float16v acc[4] = {{}, {}, {}, {}};
        for (int kk = 0; kk < KS; ++kk) {
            const uint4 av = aw[kk * 64 + lane];
            half8 a8;
            __builtin_memcpy(&a8, &av, 16);
            const int p0 = 4 * kk + 2 * h;
            int t = p0 / Lq;
            const int l = p0 - t * Lq;
            t = t < n_tx ? t : n_tx - 1;  // padded pairs carry zero taps
            const uint2* xr = xs + t * XS + (nb0 + j - l - 1 + Lq);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const uint2 x0 = xr[32 * nt], x1 = xr[32 * nt + 1];
                const uint4 bv = make_uint4(x0.x, x0.y, x1.x, x1.y);
                half8 b8;
                __builtin_memcpy(&b8, &bv, 16);
                acc[nt] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a8, b8, acc[nt], 0, 0, 0);
            }
        }

        // epilogue: lane (j, h) holds rows h and 2 + h of column 32 nt + j
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const int n = nb0 + 32 * nt + j;  // tile-relative output
            const int i = i0 + n;
            if (i >= N)
                continue;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int row = 4 * wave + 2 * q + h;
                if (row >= nu)
                    continue;
                const LinkDev& lk = links[job.link0 + row / n_rx];
                const int r = row % n_rx;
                const float yhr = acc[nt][0 + 8 * q] + acc[nt][4 + 8 * q];
                const float yhi = acc[nt][1 + 8 * q] + acc[nt][5 + 8 * q];
                const float ydr = acc[nt][2 + 8 * q] + acc[nt][6 + 8 * q];
                const float ydi = acc[nt][3 + 8 * q] + acc[nt][7 + 8 * q];
                const float a = (float)((i0 + n) % P);
                float yr = fmaf(a, ydr, yhr) * unscale[q];
                float yi = fmaf(a, ydi, yhi) * unscale[q];
                if (i0 == 0 && n < L - 1) {
                    // history terms x[n - l], l > n, of this UE (FP32)
                    for (int t = 0; t < n_tx; ++t) {
                        const float4* tr = tw + (2 * q + h) * TL + t * Lq;
                        const float2* hist = lk.hist + t * kHist;
                        for (int l = n + 1; l < L; ++l) {
                            const float4 v = tr[l];
                            const float hr = fmaf(a, v.z, v.x), hi = fmaf(a, v.w, v.y);
                            const float2 xv = hist[(L - 1) + n - l];
                            yr = fmaf(hr, xv.x, yr);
                            yr = fmaf(-hi, xv.y, yr);
                            yi = fmaf(hr, xv.y, yi);
                            yi = fmaf(hi, xv.x, yi);
                        }
                    }
                }
                const uint32_t pidx = ((uint32_t)lk.noise_base[r] + (uint32_t)i) % (uint32_t)npool;
                const float2 wv = __half22float2(noise[pidx]);
                yr = fmaf(lk.sigma, wv.x, yr);
                yi = fmaf(lk.sigma, wv.y, yi);
                reinterpret_cast<uint32_t*>(lk.y)[(int64_t)r * N + i] = encode(yr, yi, &nsat);
            }
        }
    }

    // history rewrite (first tile): the last L - 1 inputs of the call
    if (i0 == 0 && L > 1) {
        __syncthreads();  // every history read of the correction is done
        for (int e = tid; e < job.nlinks * n_tx * (L - 1); e += kBlock) {
            const int u = e / (n_tx * (L - 1));
            const int q = e - u * n_tx * (L - 1);
            const int t = q / (L - 1);
            const int kq = q - t * (L - 1);
            const LinkDev& lk = links[job.link0 + u];
            const uint32_t w = xg[(int64_t)t * N + N - (L - 1) + kq];
            lk.hist[t * kHist + kq] = make_float2((float)(int16_t)(w & 0xffffu), (float)((int32_t)w >> 16));
        }
    }
    if (__any(nsat != 0)) {
        for (int o = 32; o > 0; o >>= 1)
            nsat += __shfl_xor(nsat, o);
        if ((tid & 63) == 0)
            atomicAdd(sat, (unsigned long long)nsat);
    }
}

int dlm_lds_bytes(int L, int n_tx)
{
    const int Lq = (L + 1) & ~1;
    const int TL = n_tx * Lq;
    const int XS = kDlmBlocks * 128 + Lq;
    return ((n_tx * XS * 8 + 15) & ~15) + 4 * 4 * TL * 16 + 4 * ((TL + 3) / 4) * 64 * 16;
}

hipError_t launch_dlm(const JobDev* jobs, int njobs, int tiles_per_job, int total_tiles, int lds_bytes,
                      const LinkDev* links, const __half2* noise, int32_t npool, unsigned long long* sat,
                      hipStream_t st)
{
    if (total_tiles <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_dlm, dim3(total_tiles), dim3(kBlock), lds_bytes, st, jobs, njobs, tiles_per_job, links,
                       noise, npool, sat);
    return hipGetLastError();
}

}  // namespace tt
