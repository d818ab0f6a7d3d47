// gfx950 kernels of the channel-emulation path.
//
// k_fir: one workgroup (4 wave64) works through items; an item is one link
// (one UE direction) over one tile of T = 256 * R consecutive output samples
// of a job: a DL group (several UEs, each with its own output, possibly all
// reading the same broadcast gNB stream) or a UL group (several UEs summed
// in ascending UE order into the same registers).  A workgroup takes every
// link of its tile, then the tile gridDim.x further on, so a grid of about
// the resident workgroup count makes the kernel persistent.  For each item
// the tile's input plus the (L-1)-sample halo (from the link's resident
// history in the first tile) and the tap snapshots (or Jakes anchors)
// covering the tile are staged into LDS, then every lane accumulates R
// consecutive outputs with a register sliding window over the input: one LDS
// read of x and one broadcast LDS read of the tap pair per tap feed R complex
// multiply-adds.  The next item's input and taps are loaded into registers
// while the current one computes.  This is a short time-varying FIR, not a
// dense contraction, so it runs on the vector ALUs (no MFMA).
//
// Units: ci16 samples stay in int16 counts from input to output (both sides
// use the same 2^-12 scale, so no scaling is needed; the host passes the
// noise scale in the same units); cf32 samples are used as given.
//
// The per-sample arithmetic is fixed: for every output, taps are formed as
// h = H + a * D (a = integer offset inside the snapshot block or anchor
// interval, D the per-sample increment) and accumulated over t, then l,
// ascending, with explicit fused multiply-adds, so a result does not depend
// on the tile, the batch, the group, the grid or the prefetch setting.
#include <hip/hip_ext.h>

#include "tt_internal.h"

namespace tt {

extern __shared__ __align__(16) unsigned char g_lds[];

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

// Input sample in input units (int16 value as float for ci16; exact).
__device__ __forceinline__ float2 load_x(const void* x, int fmt, int idx)
{
    if (fmt == IQ_CI16) {
        const short2 v = reinterpret_cast<const short2*>(x)[idx];
        return make_float2((float)v.x, (float)v.y);
    }
    return reinterpret_cast<const float2*>(x)[idx];
}

__device__ __forceinline__ float2 load_tap(const void* ring, int fmt, int64_t idx)
{
    if (fmt == TAP_F16) {
        const __half2 h = reinterpret_cast<const __half2*>(ring)[idx];
        return __half22float2(h);
    }
    return reinterpret_cast<const float2*>(ring)[idx];
}

// ci16 encoding of one output given in int16 units: returns the packed
// sample and adds the number of clamped components to *sat.
__device__ __forceinline__ uint32_t encode_ci16(float2 v, int* sat)
{
    float a = rintf(v.x);
    float b = rintf(v.y);
    *sat += (a > 32767.0f || a < -32768.0f) + (b > 32767.0f || b < -32768.0f);
    a = fminf(fmaxf(a, -32768.0f), 32767.0f);
    b = fminf(fmaxf(b, -32768.0f), 32767.0f);
    return (uint32_t)(uint16_t)(int16_t)a | ((uint32_t)(uint16_t)(int16_t)b << 16);
}

__device__ __forceinline__ int store_iq(void* out, int fmt, int64_t idx, float2 v)
{
    int sat = 0;
    if (fmt == IQ_CI16)
        reinterpret_cast<uint32_t*>(out)[idx] = encode_ci16(v, &sat);
    else
        reinterpret_cast<float2*>(out)[idx] = v;
    return sat;
}

// Workgroup barrier that orders LDS only: every wave's LDS accesses before it
// are complete and visible after it.  Global stores still in flight (outputs)
// are not waited for; __syncthreads() would wait for them too.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// floor(a / b) for 0 <= a < 2^22, b >= 1, via a float reciprocal (exact in
// that range: the error of (a + 0.5) * (1/b) stays below 0.5 / b).
__device__ __forceinline__ int fdiv(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

// ---------------------------------------------------------------------------
// Tile geometry of one link inside one tile (uniform across the workgroup).
// ---------------------------------------------------------------------------
struct Geo {
    int Lp;         // taps padded to a multiple of R
    int HP;         // staged history span (>= Lp, a multiple of R and of 4)
    int S;          // LDS row length (float2) per residue class (odd: residue rows of
                    // neighbouring lanes written while staging fall in different banks)
    int nblk;       // snapshot blocks (or anchor intervals) the tile touches
    int rem0;       // offset of the tile's first output inside its first block
    int xs_bytes;   // staged input bytes
    int ts_bytes;   // staged tap-pair bytes
    int64_t kfirst; // first block index
};

// T: outputs of the item's tile (kBlock * R times the job's lane tiles).
template <int R>
__device__ __forceinline__ Geo geometry(const LinkDev& lk, int i0, int tile_len, int T)
{
    Geo g;
    g.Lp = (lk.L + R - 1) / R * R;
    g.HP = (g.Lp + 3) / 4 * 4;
    g.S = (g.HP + T) / R | 1;
    const int rr = lk.r0 + i0;
    const int q0 = rr / lk.period;
    g.kfirst = lk.k0 + q0;
    g.rem0 = rr - q0 * lk.period;
    g.nblk = (g.rem0 + tile_len - 1) / lk.period + 1;
    g.xs_bytes = lk.n_tx * R * g.S * 8;
    g.ts_bytes = g.nblk * lk.n_rx * lk.n_tx * g.Lp * 16;
    return g;
}

// Input sample i (slot-relative; negative = the link's history, zero before
// the join and past the end of the call) of transmit stream t.
__device__ __forceinline__ float2 x_at(const LinkDev& lk, int iq_fmt, int N, int t, int i)
{
    if (i >= 0)
        return i < N ? load_x(lk.x, iq_fmt, t * N + i) : make_float2(0.f, 0.f);
    if (i >= -(lk.L - 1))
        return lk.hist[t * kHist + (lk.L - 1) + i];
    return make_float2(0.f, 0.f);
}

// Four consecutive input samples i .. i + 3 of stream t; one 16- or 32-byte
// load when they lie inside the call and are aligned.
__device__ __forceinline__ void x_at4(const LinkDev& lk, int iq_fmt, int N, int t, int i, float2 (&v)[4])
{
    const int idx = t * N + i;
    if (i >= 0 && i + 3 < N && (idx & 3) == 0 && (reinterpret_cast<uintptr_t>(lk.x) & 15) == 0) {
        if (iq_fmt == IQ_CI16) {
            const int4 q = *reinterpret_cast<const int4*>(reinterpret_cast<const uint32_t*>(lk.x) + idx);
            const int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                v[j] = make_float2((float)(int16_t)(w[j] & 0xffff), (float)(w[j] >> 16));
        } else {
            const float4* p = reinterpret_cast<const float4*>(reinterpret_cast<const float2*>(lk.x) + idx);
            const float4 a = p[0], b = p[1];
            v[0] = make_float2(a.x, a.y);
            v[1] = make_float2(a.z, a.w);
            v[2] = make_float2(b.x, b.y);
            v[3] = make_float2(b.z, b.w);
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        v[j] = x_at(lk, iq_fmt, N, t, i + j);
}

// LDS position of staged relative index m (0 .. HP + T - 1) of stream t:
// residue-class layout, so that the lanes' reads of one tap step are
// consecutive words.
template <int R>
__device__ __forceinline__ int xs_pos(int t, int m, int S)
{
    return (t * R + (m % R)) * S + m / R;
}

// Stage the tile's input (+ halo) in chunks of four samples per thread.
template <int R>
__device__ void stage_x(const LinkDev& lk, const Geo& g, int iq_fmt, int N, int i0, int T, float2* xs)
{
    const int chunks = (g.HP + T) / 4;
    for (int t = 0; t < lk.n_tx; ++t) {
        for (int c = threadIdx.x; c < chunks; c += kBlock) {
            float2 v[4];
            x_at4(lk, iq_fmt, N, t, i0 - g.HP + 4 * c, v);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                xs[xs_pos<R>(t, 4 * c + j, g.S)] = v[j];
        }
    }
}

// Source offsets of tap entry e = ((blk * n_rx + r) * n_tx + t) * Lp + l in
// the ring (or caller buffer): snapshots kfirst + blk and kfirst + blk + 1.
__device__ __forceinline__ bool tap_src(const LinkDev& lk, const Geo& g, int e, float inv_rtl, float inv_lp,
                                        int64_t* s0, int64_t* s1)
{
    const int rtl = lk.n_rx * lk.n_tx * g.Lp;
    const int blk = fdiv(e, inv_rtl);
    const int q = e - blk * rtl;
    const int rt = fdiv(q, inv_lp);
    const int l = q - rt * g.Lp;
    const int per = lk.n_rx * lk.n_tx * lk.L;
    const int64_t k = g.kfirst + blk;
    const int64_t slot0 = lk.ring_cap ? k % lk.ring_cap : k - lk.kbase;
    const int64_t slot1 = lk.ring_cap ? (k + 1) % lk.ring_cap : k + 1 - lk.kbase;
    *s0 = slot0 * per + rt * lk.L + l;
    *s1 = slot1 * per + rt * lk.L + l;
    return l < lk.L;
}

// (H, D) pair: h = H + a * D per output sample.
__device__ __forceinline__ float4 tap_pair(const LinkDev& lk, float2 h, float2 hn)
{
    if (lk.mode == M_LINEAR) {
        const float s = 1.0f / (float)lk.period;
        return make_float4(h.x, h.y, (hn.x - h.x) * s, (hn.y - h.y) * s);
    }
    return make_float4(h.x, h.y, 0.f, 0.f);
}

// Stage one link's taps for the tile: the (H, D) pair of every snapshot
// block.  Jakes links come here as LINEAR links over the anchors k_anchor
// wrote for the call (snapshots K samples apart).
__device__ void stage_taps(const LinkDev& lk, const Geo& g, float4* ts)
{
    const int rtl = lk.n_rx * lk.n_tx * g.Lp;
    if (g.Lp == lk.L && lk.ring_cap == 0) {
        // unpadded taps from consecutive caller snapshots: entry e is word e
        // of the run that starts at snapshot kfirst (its next snapshot one
        // snapshot further on)
        const int64_t s0 = (g.kfirst - lk.kbase) * rtl;
        for (int e = threadIdx.x; e < g.nblk * rtl; e += kBlock) {
            const float2 h = load_tap(lk.ring, lk.tap_fmt, s0 + e);
            const float2 hn = lk.mode == M_LINEAR ? load_tap(lk.ring, lk.tap_fmt, s0 + e + rtl) : h;
            ts[e] = tap_pair(lk, h, hn);
        }
        return;
    }
    const float inv_rtl = 1.0f / (float)rtl, inv_lp = 1.0f / (float)g.Lp;
    for (int e = threadIdx.x; e < g.nblk * rtl; e += kBlock) {
        int64_t s0, s1;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (tap_src(lk, g, e, inv_rtl, inv_lp, &s0, &s1)) {
            const float2 h = load_tap(lk.ring, lk.tap_fmt, s0);
            const float2 hn = lk.mode == M_LINEAR ? load_tap(lk.ring, lk.tap_fmt, s1) : h;
            v = tap_pair(lk, h, hn);
        }
        ts[e] = v;
    }
}

// ---------------------------------------------------------------------------
// Jakes anchors of the slot's Jakes links: h_{r,t,l}(k K) for the anchors
// k0 .. k0 + count - 1 of each call, stored as fp32 snapshots
// [count][n_rx][n_tx][L] that the convolution interpolates linearly.
// One thread per (r, t, l) and group of kAnchorGroup anchors aligned to
// absolute anchor indices: the group's first anchor is evaluated exactly
// (FP64 phase reduction, then sincospi), the next ones by rotating each
// sinusoid pair's phasor by one anchor step e^{j 2 pi nu K} (from the host).
// An anchor's value depends on its index alone, whatever call uses it.  The
// pairs are summed in order m = 0 .. 7.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_anchor(const AnchorDev* __restrict__ ent, int n)
{
    // entry of this workgroup: the last one whose block0 <= blockIdx.x
    const int blk = (int)blockIdx.x;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].block0 <= blk)
            lo = mid;
        else
            hi = mid - 1;
    }
    const AnchorDev e = ent[lo];
    const int64_t g0 = e.k0 / kAnchorGroup;  // k0 >= 0
    const int ngrp = (int)((e.k0 + e.count - 1) / kAnchorGroup - g0) + 1;
    const int it = (blk - e.block0) * kBlock + (int)threadIdx.x;
    if (e.count <= 0 || it >= ngrp * e.per)
        return;
    const int gi = it / e.per;
    const int q = it - gi * e.per;  // (r * n_tx + t) * L + l
    const int64_t a_first = (g0 + gi) * kAnchorGroup;
    const int64_t PP = (int64_t)kJakesPairs * e.per;
    const double* nu = e.jakes;
    const float2* av = reinterpret_cast<const float2*>(e.jakes + PP);
    const float2* bv = av + PP;
    const float2* rv = bv + PP;
    float2 h[kAnchorGroup];
#pragma unroll
    for (int j = 0; j < kAnchorGroup; ++j)
        h[j] = make_float2(0.f, 0.f);
    const double n0 = (double)(a_first * (int64_t)e.K);
    for (int m = 0; m < kJakesPairs; ++m) {
        const int64_t o = (int64_t)m * e.per + q;
        const double pn = nu[o];
        const float2 pa = av[o], pb = bv[o], pr = rv[o];
        double c = pn * n0;
        c = c - floor(c);
        float sn, co;
        sincospif(2.0f * (float)c, &sn, &co);
#pragma unroll
        for (int j = 0; j < kAnchorGroup; ++j) {
            h[j].x = fmaf(co, pa.x, h[j].x);
            h[j].x = fmaf(sn, pb.x, h[j].x);
            h[j].y = fmaf(co, pa.y, h[j].y);
            h[j].y = fmaf(sn, pb.y, h[j].y);
            const float co2 = fmaf(co, pr.x, -(sn * pr.y));
            sn = fmaf(sn, pr.x, co * pr.y);
            co = co2;
        }
    }
#pragma unroll
    for (int j = 0; j < kAnchorGroup; ++j) {
        const int64_t a = a_first + j - e.k0;
        if (a >= 0 && a < e.count)
            e.out[a * e.per + q] = h[j];
    }
}

hipError_t launch_anchor(const AnchorDev* ent, int n, int blocks, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    if (n <= 0 || blocks <= 0)
        return hipSuccess;
    hipExtLaunchKernelGGL(k_anchor, dim3((unsigned)blocks), dim3(kBlock), 0, st, ev0, ev1, 0u, ent, n);
    return hipGetLastError();
}

// Asynchronous staging of the next work item (one link of one tile): while
// the current item computes, its raw input words and raw tap snapshots are
// copied from global memory straight into spare LDS (global_load_lds, no
// registers held); after the item's barrier, short passes unpack them into
// the staged input rows and (H, D) pairs the convolution reads.  The
// unpacked values are those of stage_x and stage_taps, bit for bit.
// Applies to items whose input lies inside the call (not the first tile,
// whose halo comes from the history) and, for taps, to dense HOLD/LINEAR
// snapshots; other items are staged synchronously.

// One 4-byte word per lane from global memory into LDS: lane l of the wave
// writes lds_wave[l].  lds_wave is the wave's base (uniform across the wave).
__device__ __forceinline__ void lds_copy_word(const uint32_t* src, uint32_t* lds_wave)
{
    __builtin_amdgcn_global_load_lds(src, lds_wave, 4, 0, 0);
}

// Words of the raw input of an item: n_tx streams of HP + T samples from
// i0 - HP in the call's storage format (ci16 one word per sample, cf32 two).
template <int IQ>
__device__ __forceinline__ int raw_x_words(const LinkDev& lk, const Geo& g, int T)
{
    return lk.n_tx * (g.HP + T) * (IQ == IQ_CI16 ? 1 : 2);
}

// Issue the copies of the raw input (samples past the end of the call are
// not copied; the unpack writes zeros there).  Requires i0 >= HP.
template <int IQ>
__device__ __forceinline__ void dma_x(const LinkDev& lk, const Geo& g, int N, int i0, int T, uint32_t* raw)
{
    constexpr int WPS = IQ == IQ_CI16 ? 1 : 2;
    const int per_stream = (g.HP + T) * WPS;
    const int total = lk.n_tx * per_stream;
    const float inv_ps = 1.0f / (float)per_stream;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(lk.x);
    const int wave_base = (int)threadIdx.x & ~63;
    for (int w0 = 0; w0 < total; w0 += kBlock) {
        const int w = w0 + (int)threadIdx.x;
        const int t = lk.n_tx > 1 ? fdiv(w, inv_ps) : 0;
        const int m = w - t * per_stream;  // word inside the stream
        const int i = i0 - g.HP + m / WPS;  // sample index in the call
        if (w < total && i < N)
            lds_copy_word(src + ((int64_t)t * N + (i0 - g.HP)) * WPS + m, raw + w0 + wave_base);
    }
}

// Unpack the copied input into the residue-class rows (zeros past the end).
template <int R, int IQ>
__device__ __forceinline__ void unpack_x(const LinkDev& lk, const Geo& g, int N, int i0, int T, const uint32_t* raw,
                                         float2* xs)
{
    constexpr int WPS = IQ == IQ_CI16 ? 1 : 2;
    const int chunks = (g.HP + T) / 4;  // per stream
    const float inv_c = 1.0f / (float)chunks;
    for (int c = threadIdx.x; c < lk.n_tx * chunks; c += kBlock) {
        const int t = lk.n_tx > 1 ? fdiv(c, inv_c) : 0;
        const int cc = c - t * chunks;
        const int i = i0 - g.HP + 4 * cc;
        const uint32_t* p = raw + ((int64_t)t * (g.HP + T) + 4 * cc) * WPS;
        float2 v[4];
        if (IQ == IQ_CI16) {
            const uint4 q = *reinterpret_cast<const uint4*>(p);
            const uint32_t wd[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                v[j] = make_float2((float)(int16_t)(wd[j] & 0xffffu), (float)((int32_t)wd[j] >> 16));
        } else {
            const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
            v[0] = make_float2(a.x, a.y);
            v[1] = make_float2(a.z, a.w);
            v[2] = make_float2(b.x, b.y);
            v[3] = make_float2(b.z, b.w);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            xs[xs_pos<R>(t, 4 * cc + j, g.S)] = i + j < N ? v[j] : make_float2(0.f, 0.f);
    }
}

// Snapshots an item's tap pairs are formed from: blocks kfirst .. kfirst +
// nblk - 1, and for LINEAR the next one.
__device__ __forceinline__ int raw_taps_words(const LinkDev& lk, const Geo& g)
{
    return (g.nblk + (lk.mode == M_LINEAR ? 1 : 0)) * lk.n_rx * lk.n_tx * lk.L * (lk.tap_fmt == TAP_F16 ? 1 : 2);
}

// Issue the copies of those snapshots: one contiguous run in a caller buffer,
// or up to two in the ring (wrapping at its end).
__device__ __forceinline__ void dma_taps(const LinkDev& lk, const Geo& g, uint32_t* raw)
{
    const int wps = lk.n_rx * lk.n_tx * lk.L * (lk.tap_fmt == TAP_F16 ? 1 : 2);
    const int nsnap = g.nblk + (lk.mode == M_LINEAR ? 1 : 0);
    const int total = nsnap * wps;
    int64_t s0;
    int run = nsnap;
    if (lk.ring_cap) {
        // slot of the first block: the link's slot of k0 plus the tile's offset
        int sl = lk.slot0 + (int)(g.kfirst - lk.k0);
        while (sl >= lk.ring_cap)
            sl -= lk.ring_cap;
        s0 = sl;
        run = min(nsnap, lk.ring_cap - sl);
    } else {
        s0 = g.kfirst - lk.kbase;
    }
    const int runw = run * wps;
    const uint32_t* ring = reinterpret_cast<const uint32_t*>(lk.ring);
    const uint32_t* first = ring + s0 * wps;
    const int wave_base = (int)threadIdx.x & ~63;
    for (int w0 = 0; w0 < total; w0 += kBlock) {
        const int w = w0 + (int)threadIdx.x;
        if (w < total)
            lds_copy_word(w < runw ? first + w : ring + (w - runw), raw + w0 + wave_base);
    }
}

// Form the (H, D) pairs from the copied snapshots, as stage_taps does.
__device__ __forceinline__ void unpack_taps(const LinkDev& lk, const Geo& g, const uint32_t* raw, float4* ts)
{
    const int rtl = lk.n_rx * lk.n_tx * g.Lp;
    const int per = lk.n_rx * lk.n_tx * lk.L;
    const float inv_rtl = 1.0f / (float)rtl, inv_lp = 1.0f / (float)g.Lp;
    for (int e = threadIdx.x; e < g.nblk * rtl; e += kBlock) {
        const int blk = fdiv(e, inv_rtl);
        const int q = e - blk * rtl;
        const int rt = fdiv(q, inv_lp);
        const int l = q - rt * g.Lp;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (l < lk.L) {
            const int o = blk * per + rt * lk.L + l;
            float2 h, hn;
            if (lk.tap_fmt == TAP_F16) {
                const __half2* hp = reinterpret_cast<const __half2*>(raw);
                h = __half22float2(hp[o]);
                hn = lk.mode == M_LINEAR ? __half22float2(hp[o + per]) : h;
            } else {
                const float2* fp = reinterpret_cast<const float2*>(raw);
                h = fp[o];
                hn = lk.mode == M_LINEAR ? fp[o + per] : h;
            }
            v = tap_pair(lk, h, hn);
        }
        ts[e] = v;
    }
}

// Accumulate one link into acc[r][q] for the lane's R consecutive outputs.
// xs: staged input in the residue-class layout (relative index m lives at
// row m % R, column m / R, so the lanes' reads of one tap step are
// consecutive words); tp: tap pairs (H, D) of the lane's snapshot block,
// [r][t][l] with l padded to Lp.  The input window slides through R
// registers: each tap step loads one new sample per lane.
template <int R, int NRX, bool INTERP, int LPC = 0>
__device__ __forceinline__ void fir_link(const float2* __restrict__ xs, const float4* __restrict__ tp, int n_tx,
                                         int Lp, int HP, int S, int tid, float a0, float (&acc)[NRX][R][2])
{
    // LPC > 0: the padded tap count is known at compile time (Lp == HP ==
    // LPC), so the tap loop unrolls fully: the input window rotates by
    // register renaming and every LDS address is an immediate offset
    if (LPC > 0) {
        Lp = LPC;
        HP = LPC;
    }
    for (int t = 0; t < n_tx; ++t) {
        const float2* xr = xs + t * R * S;
        float2 w[R];
#pragma unroll
        for (int q = 0; q < R; ++q)
            w[q] = xr[q * S + tid + HP / R];
        const float4* tpt = tp + t * Lp;
        constexpr int kUnroll = LPC > 0 ? 2 : 1;
#pragma unroll kUnroll
        for (int l0 = 0; l0 < Lp; l0 += R) {
#pragma unroll
            for (int dl = 0; dl < R; ++dl) {
                const int l = l0 + dl;
                // window slot (q - l) mod R holds x[n + q - l]; the next step needs x[n - l - 1]
                const float2 nxt = xr[(R - 1 - dl) * S + tid + (HP - l0) / R - 1];
#pragma unroll
                for (int r = 0; r < NRX; ++r) {
                    if (INTERP) {
                        const float4 hd = tpt[(size_t)r * n_tx * Lp + l];
#pragma unroll
                        for (int q = 0; q < R; ++q) {
                            const float a = a0 + (float)q;
                            const float hr = fmaf(a, hd.z, hd.x);
                            const float hi = fmaf(a, hd.w, hd.y);
                            const float2 xv = w[(q - dl + R) % R];
                            acc[r][q][0] = fmaf(hr, xv.x, acc[r][q][0]);
                            acc[r][q][0] = fmaf(-hi, xv.y, acc[r][q][0]);
                            acc[r][q][1] = fmaf(hr, xv.y, acc[r][q][1]);
                            acc[r][q][1] = fmaf(hi, xv.x, acc[r][q][1]);
                        }
                    } else {
                        const float2 h = reinterpret_cast<const float2*>(tpt + (size_t)r * n_tx * Lp + l)[0];
#pragma unroll
                        for (int q = 0; q < R; ++q) {
                            const float2 xv = w[(q - dl + R) % R];
                            acc[r][q][0] = fmaf(h.x, xv.x, acc[r][q][0]);
                            acc[r][q][0] = fmaf(-h.y, xv.y, acc[r][q][0]);
                            acc[r][q][1] = fmaf(h.x, xv.y, acc[r][q][1]);
                            acc[r][q][1] = fmaf(h.y, xv.x, acc[r][q][1]);
                        }
                    }
                }
                w[(R - 1 - dl) % R] = nxt;
            }
        }
    }
}


// Sparse top-n (Sec. III-C: only the dominant taps of each time step are
// convolved).  The selection is a property of each snapshot block, so it runs
// once per slot in k_select: per (block, r, t) group, the strength |H|^2 of
// every tap (FP64, exact squares of the stored values), the nsel strongest
// (equal strengths rank the smaller delay first), packed in ascending delay
// as (H, D) pairs with their delays.  A tile stages its blocks' selections,
// with per lane output q the staged-input offset of x[n_q - l].
// LDS layout at `base`: pairs [groups][nsel] float4 at sparse_pairs_off(ne),
// then offsets [groups][nsel][R] int, ne = groups * Lp.
__device__ __forceinline__ int sparse_pairs_off(int ne) { return (ne * 12 + 15) & ~15; }

template <int R>
__device__ void stage_sparse(const LinkDev& lk, const Geo& g, unsigned char* base)
{
    const int ngrp = g.nblk * lk.n_rx * lk.n_tx;
    const int ne = ngrp * g.Lp;
    float4* sp = reinterpret_cast<float4*>(base + sparse_pairs_off(ne));
    int* so = reinterpret_cast<int*>(base + sparse_pairs_off(ne) + ngrp * lk.nsel * 16);
    // entries of the blocks before the tile's first
    const int64_t first = (g.kfirst - lk.sk0) * lk.n_rx * lk.n_tx * lk.nsel;
    for (int e = threadIdx.x; e < ngrp * lk.nsel; e += kBlock) {
        sp[e] = lk.spairs[first + e];
        const int c = g.HP - lk.sdelay[first + e];  // staged index of x[n - l] for the lane's first output
#pragma unroll
        for (int q = 0; q < R; ++q)
            so[e * R + q] = ((c + q) % R) * g.S + (c + q) / R;
    }
}

// Lanes per group of the selection pass: L rounded up to a power of two (>= 8).
__host__ __device__ __forceinline__ int select_lanes(int L) { return L <= 8 ? 8 : L <= 16 ? 16 : L <= 32 ? 32 : 64; }

// grid: (blocks, entries), block: kBlock threads holding kSelRounds * kBlock /
// gl groups of gl lanes, lane l of a group on tap l; round i of block b takes
// the groups (b * kSelRounds + i) * kBlock / gl onward, with every round's
// loads issued before the first ranking.
// Ranking takes two passes.  The first counts, per lane, the taps whose
// strength rounded to FP32 is strictly larger: rounding is monotone, so a
// strictly larger FP32 image implies a strictly larger FP64 strength and the
// count never exceeds the lane's true rank.  The lanes counting below nsel
// therefore hold the selection; when there are exactly min(nsel, L) of them
// they are the selection.  Groups where FP32 images tie (and so more lanes
// qualify) rank again on the exact FP64 strengths.
__global__ __launch_bounds__(kBlock) void k_select(const SelectDev* __restrict__ ent)
{
    __shared__ double smag[kSelRounds][kBlock];
    __shared__ __align__(16) float smag32[kSelRounds][kBlock];
    const SelectDev& e = ent[blockIdx.y];
    const int rtn = e.n_rx * e.n_tx;
    const int per = rtn * e.L;
    const int gl = select_lanes(e.L);
    const int l = (int)threadIdx.x & (gl - 1);
    const int wl = (int)threadIdx.x & 63;  // lane in the wave; a group never straddles waves
    const unsigned long long below = wl ? (~0ull >> (64 - wl)) : 0ull;
    const unsigned long long in_grp = gl == 64 ? ~0ull : (((1ull << gl) - 1ull) << (wl - l));
    const float s = 1.0f / (float)e.period;
    // tap offsets of every round first (dead lanes read the entry's first
    // tap, which every entry has), then all loads back to back
    int64_t o0[kSelRounds], o1[kSelRounds];
#pragma unroll
    for (int i = 0; i < kSelRounds; ++i) {
        const int grp = ((int)blockIdx.x * kSelRounds + i) * (kBlock / gl) + (int)threadIdx.x / gl;
        const bool live = grp < e.nblk * rtn && l < e.L;
        o0[i] = o1[i] = (int64_t)e.s0 * per;
        if (live) {
            const int blk = rtn == 1 ? grp : grp / rtn;
            const int rt = grp - blk * rtn;
            int s0 = e.s0 + blk;
            if (e.ring_cap)
                while (s0 >= e.ring_cap)
                    s0 -= e.ring_cap;
            const int s1 = (e.ring_cap && s0 + 1 == e.ring_cap) ? 0 : s0 + 1;
            o0[i] = (int64_t)s0 * per + rt * e.L + l;
            o1[i] = e.mode == M_LINEAR ? (int64_t)s1 * per + rt * e.L + l : o0[i];
        }
    }
    float2 h[kSelRounds], hn[kSelRounds];
    if (e.tap_fmt == TAP_F16) {
        const __half2* ring = reinterpret_cast<const __half2*>(e.ring);
        __half2 a[kSelRounds], b[kSelRounds];
#pragma unroll
        for (int i = 0; i < kSelRounds; ++i) {
            a[i] = ring[o0[i]];
            b[i] = ring[o1[i]];
        }
#pragma unroll
        for (int i = 0; i < kSelRounds; ++i) {
            h[i] = __half22float2(a[i]);
            hn[i] = __half22float2(b[i]);
        }
    } else {
        const float2* ring = reinterpret_cast<const float2*>(e.ring);
#pragma unroll
        for (int i = 0; i < kSelRounds; ++i) {
            h[i] = ring[o0[i]];
            hn[i] = ring[o1[i]];
        }
    }
#pragma unroll
    for (int i = 0; i < kSelRounds; ++i) {
        const int grp = ((int)blockIdx.x * kSelRounds + i) * (kBlock / gl) + (int)threadIdx.x / gl;
        const bool live = grp < e.nblk * rtn && l < e.L;
        const double m = live ? (double)h[i].x * (double)h[i].x + (double)h[i].y * (double)h[i].y : -1.0;
        smag[i][threadIdx.x] = m;
        smag32[i][threadIdx.x] = (float)m;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSelRounds; ++i) {
        const int grp = ((int)blockIdx.x * kSelRounds + i) * (kBlock / gl) + (int)threadIdx.x / gl;
        const bool grp_live = grp < e.nblk * rtn;
        const bool live = grp_live && l < e.L;
        const double m = smag[i][threadIdx.x];
        const float m32 = smag32[i][threadIdx.x];
        // lanes l >= L of a group hold -1, below every strength, so the first
        // pass may run to L rounded up to 4 (which never passes gl)
        int gt = 0;
        if (live) {
            const float4* row = reinterpret_cast<const float4*>(&smag32[i][threadIdx.x - l]);
            const int n4 = (e.L + 3) >> 2;
#pragma unroll 4
            for (int j = 0; j < n4; ++j) {
                const float4 v = row[j];
                gt += (v.x > m32 ? 1 : 0) + (v.y > m32 ? 1 : 0) + (v.z > m32 ? 1 : 0) + (v.w > m32 ? 1 : 0);
            }
        }
        bool sel = live && gt < e.nsel;
        const bool redo = grp_live && __popcll(__ballot(sel) & in_grp) != (unsigned)min(e.nsel, e.L);
        if (__ballot(redo)) {
            if (redo && live) {
                const double* row = &smag[i][threadIdx.x - l];
                int rank = 0;
#pragma unroll 8
                for (int j = 0; j < e.L; ++j) {
                    const double mj = row[j];
                    rank += (mj > m || (mj == m && j < l)) ? 1 : 0;
                }
                sel = rank < e.nsel;
            }
        }
        // position among the group's selected lanes below this one
        const int pos = __popcll(__ballot(sel) & below & in_grp);
        // exact ranks are a permutation of 0 .. L-1, so exactly min(nsel, L)
        // lanes hold; the bound keeps non-finite taps from writing past the group
        if (sel && pos < e.nsel) {
            const float4 pair = e.mode == M_LINEAR
                                    ? make_float4(h[i].x, h[i].y, (hn[i].x - h[i].x) * s, (hn[i].y - h[i].y) * s)
                                    : make_float4(h[i].x, h[i].y, 0.f, 0.f);
            const int64_t o = (int64_t)grp * e.nsel + pos;
            e.pairs[o] = pair;
            e.delay[o] = l;
        }
    }
}

hipError_t launch_select(const SelectDev* ent, int n, int blocks, hipStream_t st)
{
    if (n <= 0 || blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_select, dim3((unsigned)blocks, (unsigned)n), dim3(kBlock), 0, st, ent);
    return hipGetLastError();
}

template <int R>
__device__ __forceinline__ const float4* sparse_pairs(const LinkDev& lk, const Geo& g, const unsigned char* base)
{
    return reinterpret_cast<const float4*>(base + sparse_pairs_off(g.nblk * lk.n_rx * lk.n_tx * g.Lp));
}

template <int R>
__device__ __forceinline__ const int* sparse_offsets(const LinkDev& lk, const Geo& g, const unsigned char* base)
{
    const int ngrp = g.nblk * lk.n_rx * lk.n_tx;
    return reinterpret_cast<const int*>(base + sparse_pairs_off(ngrp * g.Lp) + ngrp * lk.nsel * 16);
}

// Gathered FIR over the selected taps of the lane's block: sp holds the
// pairs [r][t][nsel], so the staged-input offsets [r][t][nsel][R]; per output
// the order is t, then delay, ascending, as in the dense form restricted to
// the selection.
template <int R, int NRX>
__device__ __forceinline__ void fir_sparse(const float2* __restrict__ xs, const float4* __restrict__ sp,
                                           const int* __restrict__ so, int n_tx, int nsel, int S, int tid,
                                           float a0, float (&acc)[NRX][R][2])
{
#pragma unroll
    for (int r = 0; r < NRX; ++r) {
        for (int t = 0; t < n_tx; ++t) {
            const float2* xr = xs + t * R * S + tid;
            const float4* spp = sp + (r * n_tx + t) * nsel;
            const int* sop = so + (r * n_tx + t) * nsel * R;
            for (int j = 0; j < nsel; ++j) {
                const float4 hd = spp[j];
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const float2 xv = xr[sop[j * R + q]];
                    const float a = a0 + (float)q;
                    const float hr = fmaf(a, hd.z, hd.x);
                    const float hi = fmaf(a, hd.w, hd.y);
                    acc[r][q][0] = fmaf(hr, xv.x, acc[r][q][0]);
                    acc[r][q][0] = fmaf(-hi, xv.y, acc[r][q][0]);
                    acc[r][q][1] = fmaf(hr, xv.y, acc[r][q][1]);
                    acc[r][q][1] = fmaf(hi, xv.x, acc[r][q][1]);
                }
            }
        }
    }
}

// UL finish for samples [i0, i0 + len) of one cell: (acc unless BEGIN) plus
// every group's partial in group order; END adds the noise and encodes.
__device__ int reduce_span(const ReduceDev& rd, int i0, int len, const __half2* __restrict__ noise, int32_t npool,
                           int iq_fmt)
{
    int nsat = 0;
    const int64_t gstride = (int64_t)rd.n_ant * rd.N;
    for (int e = threadIdx.x; e < rd.n_ant * len; e += kBlock) {
        const int r = e / len;
        const int i = i0 + (e - r * len);
        float2 v = make_float2(0.f, 0.f);
        if (!(rd.flags & 1))
            v = rd.acc[(int64_t)r * rd.stride + i];
        for (int g = 0; g < rd.ngroups; ++g) {
            const float2 p = rd.partial[g * gstride + (int64_t)r * rd.N + i];
            v.x += p.x;
            v.y += p.y;
        }
        if (rd.flags & 2) {
            const uint32_t p = ((uint32_t)rd.noise_base[r] + (uint32_t)i) % (uint32_t)npool;
            const float2 wv = __half22float2(noise[p]);
            v.x = fmaf(rd.sigma, wv.x, v.x);
            v.y = fmaf(rd.sigma, wv.y, v.y);
            nsat += store_iq(rd.z, iq_fmt, (int64_t)r * rd.N + i, v);
        } else {
            rd.acc[(int64_t)r * rd.stride + i] = v;
        }
    }
    return nsat;
}

// The lane's R noise samples per receive row (loaded ahead of the
// convolution so that their latency overlaps it).
template <int R, int NRX>
__device__ __forceinline__ void load_noise(__half2 (&w)[NRX][R], int ibase, const int32_t* noise_base,
                                           const __half2* __restrict__ noise, int32_t npool)
{
#pragma unroll
    for (int r = 0; r < NRX; ++r) {
        // noise_base < npool: one subtraction reduces the index when the
        // output index is below npool too (else the remainder)
        uint32_t p = (uint32_t)noise_base[r] + (uint32_t)ibase;
        if ((uint32_t)ibase < (uint32_t)npool)
            p = p >= (uint32_t)npool ? p - (uint32_t)npool : p;
        else
            p %= (uint32_t)npool;
        if (p + R <= (uint32_t)npool) {
            // the R samples are consecutive in the pool: one address
            const __half2* np = noise + p;
#pragma unroll
            for (int q = 0; q < R; ++q)
                w[r][q] = np[q];
        } else {
#pragma unroll
            for (int q = 0; q < R; ++q) {
                w[r][q] = noise[p];
                if (++p == (uint32_t)npool)
                    p = 0;
            }
        }
    }
}

// Native vector types for 16-byte non-temporal stores: outputs are written
// once and read by the caller or the next stage much later, so they stream
// past the caches.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Noise, encode and store the lane's R consecutive outputs per receive row.
template <int R, int NRX>
__device__ __forceinline__ int store_final(const float (&acc)[NRX][R][2], void* out, int N, int ibase,
                                           const __half2 (&w)[NRX][R], float sigma, int iq_fmt)
{
    int nsat = 0;
#pragma unroll
    for (int r = 0; r < NRX; ++r) {
        float2 v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const float2 wv = __half22float2(w[r][q]);
            v[q].x = fmaf(sigma, wv.x, acc[r][q][0]);
            v[q].y = fmaf(sigma, wv.y, acc[r][q][1]);
        }
        const int idx = r * N + ibase;
        if (iq_fmt == IQ_CI16) {
            uint32_t w[R];
#pragma unroll
            for (int q = 0; q < R; ++q)
                w[q] = encode_ci16(v[q], &nsat);
            uint32_t* o = reinterpret_cast<uint32_t*>(out) + idx;
            if (R == 4 && ibase + 3 < N && (idx & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
                __builtin_nontemporal_store(u32x4{w[0], w[1 % R], w[2 % R], w[3 % R]}, reinterpret_cast<u32x4*>(o));
            } else {
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (ibase + q < N)
                        o[q] = w[q];
            }
        } else {
            float2* o = reinterpret_cast<float2*>(out) + idx;
            if (R % 2 == 0 && ibase + R - 1 < N && (idx & 1) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
                // the lane's R outputs are contiguous: 16-byte stores
#pragma unroll
                for (int q = 0; q + 1 < R; q += 2)
                    __builtin_nontemporal_store(f32x4{v[q].x, v[q].y, v[q + 1].x, v[q + 1].y},
                                                reinterpret_cast<f32x4*>(o + q));
            } else {
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (ibase + q < N)
                        o[q] = v[q];
            }
        }
    }
    return nsat;
}

// End of a UL job's tile, once every link has accumulated: the sum plus the
// cell noise, encoded (J_FINAL), or the group's FP32 partial (J_PARTIAL),
// which the last group of the tile also reduces when the job carries a
// reduction (fused UL sum).
template <int R, int NRX>
__device__ int ul_epilogue(const JobDev& job, int tile, int i0, int N, int ibase, bool live,
                           const float (&acc)[NRX][R][2], const ReduceDev* __restrict__ reds,
                           const __half2* __restrict__ noise, int32_t npool, int iq_fmt)
{
    constexpr int T = kBlock * R;
    const int tid = threadIdx.x;
    int nsat = 0;
    if (job.kind == J_FINAL) {
        if (live) {
            __half2 wu[NRX][R];
            load_noise<R, NRX>(wu, ibase, job.noise_base, noise, npool);
            nsat += store_final<R, NRX>(acc, job.out, N, ibase, wu, job.sigma, iq_fmt);
        }
        return nsat;
    }
    float2* out = reinterpret_cast<float2*>(job.out);
    if (live) {
#pragma unroll
        for (int r = 0; r < NRX; ++r)
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int i = ibase + q;
                if (i < N)
                    out[r * N + i] = make_float2(acc[r][q][0], acc[r][q][1]);
            }
    }
    if (job.red >= 0) {
        // The last group to finish this tile sums every group's partial in
        // group order (fixed), adds the cell noise and stores.  Every lane
        // releases its own partial stores at device scope before the tile
        // counter moves, and the last group acquires before reading the
        // others'.
        __shared__ int s_last;
        __threadfence();
        __syncthreads();
        if (tid == 0) {
            const ReduceDev& rd = reds[job.red];
            const unsigned old = atomicAdd(&rd.counters[tile], 1u);
            const int last = old == (unsigned)(rd.ngroups - 1);
            if (last)
                atomicExch(&rd.counters[tile], 0u);
            s_last = last;
        }
        __syncthreads();
        if (s_last) {
            __threadfence();
            nsat += reduce_span(reds[job.red], i0, min(T, N - i0), noise, npool, iq_fmt);
        }
    }
    return nsat;
}

// Job of a tile: direct when every job has the same number of tiles, else a
// binary search over the jobs' first tiles.
__device__ __forceinline__ int job_of(const JobDev* __restrict__ jobs, int njobs, int tiles_per_job, int tile)
{
    if (tiles_per_job > 0)
        return tile / tiles_per_job;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= tile)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One work item: link `link` of job `job` over tile `tile` (tile < 0: none).
struct Item {
    int tile, job, link;
};

// Items of a workgroup: every link of its tile, then the tile gridDim.x
// further on (a grid smaller than the tile count makes the kernel persistent).
__device__ __forceinline__ Item next_item(const Item& c, const JobDev* __restrict__ jobs, int njobs,
                                          int tiles_per_job, int total_tiles)
{
    Item n = c;
    if (c.link + 1 < jobs[c.job].nlinks) {
        n.link = c.link + 1;
        return n;
    }
    n.link = 0;
    n.tile = c.tile + (int)gridDim.x;
    if (n.tile >= total_tiles) {
        n.tile = -1;
        return n;
    }
    n.job = job_of(jobs, njobs, tiles_per_job, n.tile);
    return n;
}

// s_waitcnt vmcnt(0) alone (expcnt and lgkmcnt left at their maxima):
// every vector memory operation of the wave issued so far has completed.
__device__ __forceinline__ void wait_vm_all() { __builtin_amdgcn_s_waitcnt(0x0f70); }

// SUBT: the launch has DL jobs of several lane tiles per item (a separate
// instantiation, so that one-tile launches keep the registers the loop over
// lane tiles would take).
template <int R, int NRX, int IQ, bool PF, bool SUBT>
// Six resident waves per SIMD for the single-row shapes at up to four
// outputs per lane (they fit in 80 VGPRs without spilling): the kernel is
// bound by how many waves have a multiply-add ready, not by any one wave's
// stream.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(R <= 4 && NRX == 1 ? 6 : 1, 8)))
void k_fir(const JobDev* __restrict__ jobs, int njobs, int tiles_per_job, int total_tiles,
           const LinkDev* __restrict__ links, const ReduceDev* __restrict__ reds,
           const __half2* __restrict__ noise, int32_t npool, unsigned long long* __restrict__ sat, int raw_off,
           int rawx_bytes, int rawt_bytes)
{
    constexpr int TL = kBlock * R;  // outputs of one lane tile
    const int tid = threadIdx.x;
    if ((int)blockIdx.x >= total_tiles)
        return;
    int nsat = 0;
    float acc[NRX][R][2];

    float2* const xs = reinterpret_cast<float2*>(g_lds);
    uint32_t* const raw_x = reinterpret_cast<uint32_t*>(g_lds + raw_off);
    uint32_t* const raw_t = reinterpret_cast<uint32_t*>(g_lds + raw_off + rawx_bytes);
    auto tap_buf = [&](const Geo& g) { return reinterpret_cast<float4*>(g_lds + g.xs_bytes); };
    auto sel_buf = [&](const Geo& g) { return g_lds + g.xs_bytes + g.ts_bytes; };  // sparse
    auto link_of = [&](const Item& it) -> const LinkDev& { return links[jobs[it.job].link0 + it.link]; };
    // a job's items cover sub lane tiles each
    auto tile_of = [&](const Item& it) { return SUBT ? TL * jobs[it.job].sub : TL; };
    auto first_of = [&](const Item& it) { return (it.tile - jobs[it.job].tile0) * tile_of(it); };
    auto geo_of = [&](const Item& it) {
        const int i0 = first_of(it);
        const int T = tile_of(it);
        return geometry<R>(link_of(it), i0, min(T, jobs[it.job].N - i0), T);
    };
    // DL UEs of one group share the broadcast input, except in the first
    // tile, whose halo comes from each UE's own history.
    auto shares_x = [&](const Item& it) { return it.link > 0 && jobs[it.job].shared_x && first_of(it) > 0; };

    // a link's taps for the tile: every (H, D) pair, or the sparse selection
    auto stage_link_taps = [&](const LinkDev& lk, const Geo& gg) {
        if (lk.nsel > 0)
            stage_sparse<R>(lk, gg, sel_buf(gg));
        else
            stage_taps(lk, gg, tap_buf(gg));
    };

    Item cur{(int)blockIdx.x, job_of(jobs, njobs, tiles_per_job, (int)blockIdx.x), 0};
    Geo g = geo_of(cur);
    stage_x<R>(link_of(cur), g, IQ, jobs[cur.job].N, first_of(cur), tile_of(cur), xs);
    stage_link_taps(link_of(cur), g);
    Item nxt = next_item(cur, jobs, njobs, tiles_per_job, total_tiles);
    lds_barrier();

    for (;;) {
        const JobDev& job = jobs[cur.job];
        const LinkDev& lk = link_of(cur);
        const int N = job.N;
        const int i0 = first_of(cur);
        const int ibase0 = i0 + tid * R;  // the lane's first output in the item's first lane tile

        // the next item's raw input and taps start their way into LDS now
        Geo gn = g;
        bool dx = false, dt = false, wx = false;
        if (nxt.tile >= 0) {
            gn = geo_of(nxt);
            const LinkDev& nl = link_of(nxt);
            wx = !shares_x(nxt);
            if constexpr (PF) {
                const int ni0 = first_of(nxt);
                const int nT = tile_of(nxt);
                dx = wx && ni0 >= gn.HP && raw_x_words<IQ>(nl, gn, nT) * 4 <= rawx_bytes;
                dt = nl.nsel == 0 && raw_taps_words(nl, gn) * 4 <= rawt_bytes;
                if (dx)
                    dma_x<IQ>(nl, gn, jobs[nxt.job].N, ni0, nT, raw_x);
                if (dt)
                    dma_taps(nl, gn, raw_t);
            }
        }

        if (cur.link == 0 || job.kind == J_DL) {
#pragma unroll
            for (int r = 0; r < NRX; ++r)
#pragma unroll
                for (int q = 0; q < R; ++q)
                    acc[r][q][0] = acc[r][q][1] = 0.f;
        }

        // history rewrite (first tile): the last L - 1 inputs of this call
        if (i0 == 0 && lk.write_hist && lk.L > 1) {
            for (int e = tid; e < lk.n_tx * (lk.L - 1); e += kBlock) {
                const int t = e / (lk.L - 1);
                const int k = e - t * (lk.L - 1);
                const int s = N - (lk.L - 1) + k;
                const float2 v = s >= 0 ? load_x(lk.x, IQ, t * N + s) : xs[xs_pos<R>(t, s + g.HP, g.S)];
                lk.hist[t * kHist + k] = v;
            }
        }

        // the item's lane tiles in order (a UL item has one): lane tid of tile
        // s computes outputs i0 + s * TL + tid * R .. + R - 1, which sit in
        // column tid + s * kBlock of the staged rows
        const int nsub = SUBT ? job.sub : 1;
        for (int s = 0; s < nsub; ++s) {
            if (SUBT && s > 0) {
#pragma unroll
                for (int r = 0; r < NRX; ++r)
#pragma unroll
                    for (int q = 0; q < R; ++q)
                        acc[r][q][0] = acc[r][q][1] = 0.f;
            }
            const int col = tid + s * kBlock;
            const int ibase = ibase0 + s * TL;
            const bool live = ibase < N;
            __half2 wn[NRX][R];
            if (job.kind == J_DL && live)
                load_noise<R, NRX>(wn, ibase, lk.noise_base, noise, npool);
            if (live) {
                const int rem = g.rem0 + col * R;
                const int blk = rem / lk.period;
                const float a0 = (float)(rem - blk * lk.period);
                const float4* tp = tap_buf(g) + (size_t)blk * NRX * lk.n_tx * g.Lp;
                if (lk.nsel > 0)
                    fir_sparse<R, NRX>(xs,
                                       sparse_pairs<R>(lk, g, sel_buf(g)) + (size_t)blk * NRX * lk.n_tx * lk.nsel,
                                       sparse_offsets<R>(lk, g, sel_buf(g)) +
                                           (size_t)blk * NRX * lk.n_tx * lk.nsel * R,
                                       lk.n_tx, lk.nsel, g.S, col, a0, acc);
                else if (NRX == 1 && lk.mode != M_HOLD && g.Lp == 32 && g.HP == 32)
                    fir_link<R, NRX, true, 32>(xs, tp, lk.n_tx, g.Lp, g.HP, g.S, col, a0, acc);
                else if (lk.mode != M_HOLD)
                    fir_link<R, NRX, true>(xs, tp, lk.n_tx, g.Lp, g.HP, g.S, col, a0, acc);
                else
                    fir_link<R, NRX, false>(xs, tp, lk.n_tx, g.Lp, g.HP, g.S, col, a0, acc);
            }
            // the copies into LDS (and the noise loads) are complete: waited
            // for here, before the first output stores, so the barrier below
            // does not wait for the stores
            if (PF && s == 0 && (dx || dt))
                wait_vm_all();

            if (job.kind == J_DL) {
                // each DL UE of the group has its own output
                if (live)
                    nsat += store_final<R, NRX>(acc, lk.y, N, ibase, wn, lk.sigma, IQ);
            } else if (cur.link == job.nlinks - 1) {
                nsat += ul_epilogue<R, NRX>(job, cur.tile - job.tile0, i0, N, ibase, live, acc, reds, noise, npool,
                                            IQ);
            }
        }

        if (nxt.tile < 0)
            break;
        // every wave is done reading this item's LDS data and its copies for
        // the next item have landed (outputs still in flight are not waited for)
        lds_barrier();
        const LinkDev& nl = link_of(nxt);
        if (dx)
            unpack_x<R, IQ>(nl, gn, jobs[nxt.job].N, first_of(nxt), tile_of(nxt), raw_x, xs);
        else if (wx)
            stage_x<R>(nl, gn, IQ, jobs[nxt.job].N, first_of(nxt), tile_of(nxt), xs);
        if (dt)
            unpack_taps(nl, gn, raw_t, tap_buf(gn));
        else
            stage_link_taps(nl, gn);
        lds_barrier();
        cur = nxt;
        g = gn;
        nxt = next_item(cur, jobs, njobs, tiles_per_job, total_tiles);
    }
    // one atomic per wave that clamped anything
    if (__any(nsat != 0)) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            nsat += __shfl_xor(nsat, o);
        if ((tid & 63) == 0)
            atomicAdd(sat, (unsigned long long)nsat);
    }
}

template <int R, int NRX, int IQ, bool PF, bool SUBT>
static hipError_t launch_fir_s(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                               const ReduceDev* reds, const __half2* noise, int32_t npool,
                               unsigned long long* sat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    if (ev0 || ev1)
        hipExtLaunchKernelGGL((k_fir<R, NRX, IQ, PF, SUBT>), dim3(s.grid), dim3(kBlock), s.lds_bytes, st, ev0, ev1, 0u,
                              jobs, njobs, s.tiles_per_job, s.total_tiles, links, reds, noise, npool, sat,
                              s.raw_off, s.rawx_bytes, s.rawt_bytes);
    else
        hipLaunchKernelGGL((k_fir<R, NRX, IQ, PF, SUBT>), dim3(s.grid), dim3(kBlock), s.lds_bytes, st, jobs, njobs,
                           s.tiles_per_job, s.total_tiles, links, reds, noise, npool, sat, s.raw_off, s.rawx_bytes,
                           s.rawt_bytes);
    return hipGetLastError();
}

template <int R, int NRX, int IQ, bool PF>
static hipError_t launch_fir_t(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                               const ReduceDev* reds, const __half2* noise, int32_t npool,
                               unsigned long long* sat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    // items of several lane tiles come with synchronous staging and R <= 4
    // only (the host keeps one tile otherwise)
    if constexpr (!PF && R <= 4) {
        if (s.subtiles)
            return launch_fir_s<R, NRX, IQ, PF, true>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
    } else {
        if (s.subtiles)
            return hipErrorInvalidValue;
    }
    return launch_fir_s<R, NRX, IQ, PF, false>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
}

template <int R, int IQ, bool PF>
static hipError_t launch_fir_n(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                               const ReduceDev* reds, const __half2* noise, int32_t npool,
                               unsigned long long* sat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    switch (s.nrx) {
    case 1: return launch_fir_t<R, 1, IQ, PF>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
    case 2: return launch_fir_t<R, 2, IQ, PF>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
    case 3: return launch_fir_t<R, 3, IQ, PF>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
    case 4: return launch_fir_t<R, 4, IQ, PF>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

template <int R>
static hipError_t launch_fir_r(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                               const ReduceDev* reds, const __half2* noise, int32_t npool, int iq_fmt,
                               unsigned long long* sat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    if (iq_fmt == IQ_CI16)
        return s.prefetch ? launch_fir_n<R, IQ_CI16, true>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1)
                          : launch_fir_n<R, IQ_CI16, false>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
    return s.prefetch ? launch_fir_n<R, IQ_CF32, true>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1)
                      : launch_fir_n<R, IQ_CF32, false>(s, jobs, njobs, links, reds, noise, npool, sat, st, ev0, ev1);
}

hipError_t launch_fir(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                      const ReduceDev* reds, const __half2* noise, int32_t npool, int iq_fmt,
                      unsigned long long* sat, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1)
{
    if (s.total_tiles <= 0 || s.grid <= 0)
        return hipSuccess;
    switch (s.R) {
    case 1: return launch_fir_r<1>(s, jobs, njobs, links, reds, noise, npool, iq_fmt, sat, st, ev0, ev1);
    case 2: return launch_fir_r<2>(s, jobs, njobs, links, reds, noise, npool, iq_fmt, sat, st, ev0, ev1);
    case 4: return launch_fir_r<4>(s, jobs, njobs, links, reds, noise, npool, iq_fmt, sat, st, ev0, ev1);
    case 8: return launch_fir_r<8>(s, jobs, njobs, links, reds, noise, npool, iq_fmt, sat, st, ev0, ev1);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// UL second pass: fixed-order sum over groups, cell noise, encode.
// grid: (ceil(max_n / 64), max_ant, nred) of single waves, which spreads a
// slot's few hundred kilobytes of output over every compute unit
// ---------------------------------------------------------------------------
constexpr int kRedBlock = 64;

__global__ __launch_bounds__(kRedBlock) void k_reduce(const ReduceDev* __restrict__ reds,
                                                      const __half2* __restrict__ noise, int32_t npool,
                                                      int iq_fmt, unsigned long long* __restrict__ sat)
{
    const ReduceDev& rd = reds[blockIdx.z];
    const int r = blockIdx.y;
    const int i = blockIdx.x * kRedBlock + threadIdx.x;
    if (r >= rd.n_ant || i >= rd.N)
        return;
    // noise first: its load overlaps the partial sums
    float2 wv = make_float2(0.f, 0.f);
    if (rd.flags & 2)
        wv = __half22float2(noise[((uint32_t)rd.noise_base[r] + (uint32_t)i) % (uint32_t)npool]);
    float2 v = make_float2(0.f, 0.f);
    if (!(rd.flags & 1))
        v = rd.acc[(int64_t)r * rd.stride + i];
    const int64_t gstride = (int64_t)rd.n_ant * rd.N;
    const float2* pp = rd.partial + (int64_t)r * rd.N + i;
    // eight independent loads in flight, summed in group order
    int g = 0;
    for (; g + 8 <= rd.ngroups; g += 8) {
        float2 p[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            p[k] = pp[(g + k) * gstride];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v.x += p[k].x;
            v.y += p[k].y;
        }
    }
    for (; g < rd.ngroups; ++g) {
        const float2 p = pp[g * gstride];
        v.x += p.x;
        v.y += p.y;
    }
    if (rd.flags & 2) {
        v.x = fmaf(rd.sigma, wv.x, v.x);
        v.y = fmaf(rd.sigma, wv.y, v.y);
        const int ns = store_iq(rd.z, iq_fmt, (int64_t)r * rd.N + i, v);
        if (ns)
            atomicAdd(sat, (unsigned long long)ns);
    } else {
        rd.acc[(int64_t)r * rd.stride + i] = v;
    }
}

hipError_t launch_reduce(const ReduceDev* red, int nred, int max_n, int max_ant, const __half2* noise,
                         int32_t npool, int iq_fmt, unsigned long long* sat, hipStream_t st)
{
    if (nred <= 0 || max_n <= 0)
        return hipSuccess;
    dim3 grid((max_n + kRedBlock - 1) / kRedBlock, max_ant, nred);
    hipLaunchKernelGGL(k_reduce, grid, dim3(kRedBlock), 0, st, red, noise, npool, iq_fmt, sat);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tap ingest from device sources into rings. grid: (chunks, n entries)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_ingest(const IngestDev* __restrict__ ent)
{
    const IngestDev& e = ent[blockIdx.y];
    const int64_t total = (int64_t)e.count * e.per;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kBlock) {
        const int64_t s = i / e.per;
        const int64_t j = i - s * e.per;
        const int64_t dst = ((e.k0 + s) % e.cap) * e.per + j;
        if (e.bytes_per_tap == 8)
            reinterpret_cast<float2*>(e.ring)[dst] = reinterpret_cast<const float2*>(e.src)[i];
        else
            reinterpret_cast<uint32_t*>(e.ring)[dst] = reinterpret_cast<const uint32_t*>(e.src)[i];
    }
}

hipError_t launch_ingest(const IngestDev* ent, int n, int64_t max_taps, hipStream_t st)
{
    if (n <= 0 || max_taps <= 0)
        return hipSuccess;
    int64_t chunks = (max_taps + kBlock - 1) / kBlock;
    if (chunks > 1024)
        chunks = 1024;
    hipLaunchKernelGGL(k_ingest, dim3((unsigned)chunks, n), dim3(kBlock), 0, st, ent);
    return hipGetLastError();
}

// Descriptor upload: the kernel reads pinned host memory and writes device
// memory, which keeps the upload on the compute queue.
__global__ __launch_bounds__(kBlock) void k_copy16(int4* __restrict__ dst, const int4* __restrict__ src, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n)
        dst[i] = src[i];
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t st)
{
    const int64_t n = (bytes + 15) / 16;
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       reinterpret_cast<int4*>(dst), reinterpret_cast<const int4*>(src), n);
    return hipGetLastError();
}

__global__ void k_zero(uint32_t* p, int64_t words)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st)
{
    const int64_t words = bytes / 4;
    if (words <= 0)
        return hipSuccess;
    int64_t blocks = (words + kBlock - 1) / kBlock;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(kBlock), 0, st, reinterpret_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

}  // namespace tt
