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
// 32-row matrix tile) and all four 32-sample column tiles of each block and,
// after the shared input is staged, works without workgroup barriers: it
// stages its rows' taps, splits each into f16 parts once, assembles its A
// operand table in LDS, prefetches the next block's snapshot and runs
// 4 x KS MFMAs per block in two passes of two column tiles (one A read per
// two MFMAs); the input tile is staged once for all waves.  Matrix layout of one wave and block:
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
    const int r0 = l0.r0;  // the group's clock offset inside its snapshot block (a multiple of 128)
    const bool linear = l0.mode == M_LINEAR;
    const int nu = job.nlinks * n_rx;  // (UE, rx) rows in use, <= 16
    const int Lq = (L + 1) & ~1;
    const int TL = n_tx * Lq;            // (tx, tap) entries per row
    const int KS = (TL + 3) / 4;         // MFMA depth steps (<= 8)
    const int XS = TM + Lq;
    uint2* xs = reinterpret_cast<uint2*>(g_lds_m);
    float4* tw = reinterpret_cast<float4*>(g_lds_m + ((n_tx * XS * 8 + 15) & ~15)) + wave * 4 * TL;
    uint4* sw = reinterpret_cast<uint4*>(g_lds_m + ((n_tx * XS * 8 + 15) & ~15) + 4 * 4 * TL * 16) + wave * 4 * TL;
    uint4* aw = reinterpret_cast<uint4*>(g_lds_m + ((n_tx * XS * 8 + 15) & ~15) + 2 * 4 * 4 * TL * 16) + wave * KS * 64;
    // per (UE, rx) row: output, noise base, noise scale, history (rows < nu)
    __shared__ uint32_t* s_y[16];
    __shared__ const float2* s_hist[16];
    __shared__ int32_t s_nb[16];
    __shared__ float s_sig[16];
    if (tid < 16 && tid < nu) {
        const LinkDev& lk = links[job.link0 + tid / n_rx];
        const int r = tid % n_rx;
        s_y[tid] = reinterpret_cast<uint32_t*>(lk.y) + (int64_t)r * N;
        s_hist[tid] = lk.hist;
        s_nb[tid] = lk.noise_base[r];
        s_sig[tid] = lk.sigma;
    }
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
    // the row's snapshot source, read once (outputs are stored through
    // pointers the compiler cannot tell apart from the descriptors)
    const int64_t k0_me = lk_me.k0, kbase_me = lk_me.kbase;
    const int32_t cap_me = lk_me.ring_cap;
    const int32_t per_me = lk_me.n_rx * lk_me.n_tx * lk_me.L;
    const bool f16_me = lk_me.tap_fmt == TAP_F16;
    const void* const ring_me = lk_me.ring;
    auto load = [&](int64_t koff_q, float2 (&v)[2]) {
        const int64_t k = k0_me + koff_q;
        const int64_t slot = cap_me ? k % cap_me : k - kbase_me;
        const int64_t base = slot * per_me;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            v[m] = make_float2(0.f, 0.f);
            if (ok_me[m]) {
                const int64_t idx = base + off_me[m];
                v[m] = f16_me ? __half22float2(reinterpret_cast<const __half2*>(ring_me)[idx])
                              : reinterpret_cast<const float2*>(ring_me)[idx];
            }
        }
    };
    float2 sa[2], sb[2], pf[2];
    int64_t have = -1, pf_k = -1;
    float unscale[2] = {1.f, 1.f};

    __syncthreads();  // shared input and row descriptors staged; from here on each wave works alone

    // Within a wave, LDS accesses complete in program order, so the wave's
    // own tap, split and operand tables need no workgroup barrier; the code
    // motion barrier keeps the compiler from moving reads above writes.
    auto wave_sync = [] { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); __builtin_amdgcn_wave_barrier(); };
    for (int b = 0; b < kDlmBlocks; ++b) {
        const int nb0 = b * 128;
        if (i0 + nb0 >= N)
            break;
        const int64_t koff = ((int64_t)r0 + i0 + nb0) / P;
        const bool rebuild = koff != have;
        // the block's noise samples, loaded now so that their latency hides
        // behind the operand build and the contraction
        __half2 wn[2][2][2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int row = 4 * wave + 2 * q + h;
            const uint32_t nb = row < nu ? ((uint32_t)s_nb[row] + (uint32_t)(i0 + nb0)) % (uint32_t)npool : 0u;
#pragma unroll
            for (int pass = 0; pass < 2; ++pass)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const int nn = 64 * pass + 32 * c + j;
                    uint32_t pidx = nb + (uint32_t)nn;
                    if (pidx >= (uint32_t)npool)
                        pidx %= (uint32_t)npool;
                    wn[pass][c][q] = (row < nu && i0 + nb0 + nn < N) ? noise[pidx] : __half2{};
                }
        }
        if (rebuild) {
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
        }
        // prefetch the snapshot the next block adds; it lands while this
        // block builds its operands and contracts
        if (b + 1 < kDlmBlocks && i0 + nb0 + 128 < N) {
            const int64_t kn = ((int64_t)r0 + i0 + nb0 + 128) / P;
            const int64_t want = linear ? kn + 1 : kn;
            if (kn != koff && pf_k != want) {
                pf_k = want;
                load(pf_k, pf);
            }
        }
        if (rebuild) {
            wave_sync();  // the previous block's tables are no longer read by this wave
            const float inv_p = 1.0f / (float)P;
            float mx = 0.f;
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
                    mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
                }
            }
            // row maxima: the 16 lanes of a row reduce, lane 16 u then holds row u's
#pragma unroll
            for (int o = 8; o > 0; o >>= 1)
                mx = fmaxf(mx, __shfl_xor(mx, o));
            // power-of-two scales: largest component in [2^14, 2^15)
            auto scale_of = [](float m, float* sc, float* usc) {
                int ex = 0;
                if (m > 0.f)
                    (void)frexpf(m, &ex);
                const int sh = m > 0.f ? min(15 - ex, 126) : 0;
                *sc = ldexpf(1.0f, sh);
                *usc = ldexpf(1.0f, -sh);
            };
            float sc_me, tmp;
            scale_of(mx, &sc_me, &tmp);
            scale_of(__shfl(mx, 16 * h), &tmp, &unscale[0]);        // row h
            scale_of(__shfl(mx, 16 * (2 + h)), &tmp, &unscale[1]);  // row 2 + h
            // f16 splits of the lane's scaled taps, once per tap: per entry
            // (H re hi|lo, H im hi|lo, D re hi|lo, D im hi|lo)
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                const int q = (lane & 15) + 16 * m;
                if (q < TL) {
                    const float4 v = tw[u_me * TL + q];
                    const float f[4] = {v.x * sc_me, v.y * sc_me, v.z * sc_me, v.w * sc_me};
                    uint32_t w[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const _Float16 hi = (_Float16)f[c];
                        const _Float16 lo = (_Float16)(f[c] - (float)hi);
                        w[c] = (uint32_t)__builtin_bit_cast(uint16_t, hi) |
                               ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
                    }
                    sw[u_me * TL + q] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
            wave_sync();
            // A operand table of the wave: entry (kk, lane) = row i = j, half h.
            // Row i takes, per tap and input part, the split part s_h of the
            // coefficient: out re <- (re, -im), out im <- (im, re).
            {
                const int i = j;
                const int u = 2 * (i >> 4) + ((i >> 2) & 1);
                const int shift = ((i >> 3) & 1) * 16;  // split part s_h
                const int hd = (i >> 1) & 1;            // c = i % 4 = 2 hd + cout
                const int cout = i & 1;
                const uint32_t neg = cout ? 0u : 0x80008000u;  // -im for the real output
                int t_a = 0, l_a = 2 * h;
                for (int kk = 0; kk < KS; ++kk) {
                    uint32_t d[4];
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        // taps l_a + 1 (elements 0..3) then l_a (elements 4..7)
                        const int l = l_a + 1 - q;
                        uint32_t wre = 0u, wim = 0u;
                        if (t_a < n_tx) {
                            const uint4 v = sw[u * TL + t_a * Lq + l];
                            wre = hd ? v.z : v.x;
                            wim = hd ? v.w : v.y;
                        }
                        const uint32_t re = (wre >> shift) & 0xffffu, im = (wim >> shift) & 0xffffu;
                        const uint32_t a0 = cout ? im : re;  // input re
                        const uint32_t a1 = cout ? re : im;  // input im (negated for the real output)
                        d[2 * q + 0] = a0 | (a0 << 16);
                        d[2 * q + 1] = (a1 | (a1 << 16)) ^ neg;
                    }
                    aw[kk * 64 + lane] = make_uint4(d[0], d[1], d[2], d[3]);
                    l_a += 4;
                    while (l_a >= Lq) {
                        l_a -= Lq;
                        ++t_a;
                    }
                }
            }
            wave_sync();
        }

        // contraction and epilogue in two passes of two 32-sample column tiles
        const int a_blk = (int)(((int64_t)r0 + i0 + nb0) % P);  // offset of the block's first output in its snapshot block
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            float16v acc[2] = {{}, {}};
            int t_k = 0, l_k = 2 * h;  // (t, l) of pair 4 kk + 2 h (Lq even)
            for (int kk = 0; kk < KS; ++kk) {
                const uint4 av = aw[kk * 64 + lane];
                half8 a8;
                __builtin_memcpy(&a8, &av, 16);
                const int t = t_k < n_tx ? t_k : n_tx - 1;  // padded pairs carry zero taps
                const uint2* xr = xs + t * XS + (nb0 + 64 * pass + j - l_k - 1 + Lq);
                l_k += 4;
                while (l_k >= Lq) {
                    l_k -= Lq;
                    ++t_k;
                }
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const uint2 x0 = xr[32 * c], x1 = xr[32 * c + 1];
                    const uint4 bv = make_uint4(x0.x, x0.y, x1.x, x1.y);
                    half8 b8;
                    __builtin_memcpy(&b8, &bv, 16);
                    acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a8, b8, acc[c], 0, 0, 0);
                }
            }

            // epilogue: lane (j, h) holds rows h and 2 + h of its column
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int nn = 64 * pass + 32 * c + j;  // block-relative output
                const int n = nb0 + nn;                  // tile-relative output
                const int i = i0 + n;
                if (i >= N)
                    continue;
                const float a = (float)(a_blk + nn);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int row = 4 * wave + 2 * q + h;
                    if (row >= nu)
                        continue;
                    const float yhr = acc[c][0 + 8 * q] + acc[c][4 + 8 * q];
                    const float yhi = acc[c][1 + 8 * q] + acc[c][5 + 8 * q];
                    const float ydr = acc[c][2 + 8 * q] + acc[c][6 + 8 * q];
                    const float ydi = acc[c][3 + 8 * q] + acc[c][7 + 8 * q];
                    float yr = fmaf(a, ydr, yhr) * unscale[q];
                    float yi = fmaf(a, ydi, yhi) * unscale[q];
                    if (i0 == 0 && n < L - 1) {
                        // history terms x[n - l], l > n, of this UE (FP32)
                        const float2* hist0 = s_hist[row];
#pragma unroll 1
                        for (int t = 0; t < n_tx; ++t) {
                            const float4* tr = tw + (2 * q + h) * TL + t * Lq;
                            const float2* hist = hist0 + t * kHist;
#pragma unroll 1
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
                    const float2 wv = __half22float2(wn[pass][c][q]);
                    const float sg = s_sig[row];
                    yr = fmaf(sg, wv.x, yr);
                    yi = fmaf(sg, wv.y, yi);
                    s_y[row][i] = encode(yr, yi, &nsat);
                }
            }
        }
    }

    // history rewrite (first tile): the last L - 1 inputs of the call
    if (i0 == 0 && L > 1) {
        __syncthreads();  // every wave's history reads of the correction are done
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
    return ((n_tx * XS * 8 + 15) & ~15) + 2 * 4 * 4 * TL * 16 + 4 * ((TL + 3) / 4) * 64 * 16;
}

hipError_t launch_dlm(const JobDev* jobs, int njobs, int tiles_per_job, int total_tiles, int lds_bytes,
                      const LinkDev* links, const __half2* noise, int32_t npool, unsigned long long* sat,
                      hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    if (total_tiles <= 0)
        return hipSuccess;
    if (ev0 || ev1)
        hipExtLaunchKernelGGL(k_dlm, dim3(total_tiles), dim3(kBlock), lds_bytes, st, ev0, ev1, 0u, jobs, njobs,
                              tiles_per_job, links, noise, npool, sat);
    else
        hipLaunchKernelGGL(k_dlm, dim3(total_tiles), dim3(kBlock), lds_bytes, st, jobs, njobs, tiles_per_job,
                           links, noise, npool, sat);
    return hipGetLastError();
}

}  // namespace tt
