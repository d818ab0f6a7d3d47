// gfx950 kernels of the channel-emulation path.
//
// k_fir: one workgroup (4 wave64) computes one tile of T = 256 * R consecutive
// output samples of one job: a DL UE (one link) or a UL group (several links
// summed in ascending UE order into the same registers).  Per link it stages
// the tile's input plus the (L-1)-sample halo into LDS as cf32 (the halo of
// the first tile comes from the link's resident history), stages the tap
// snapshots (or Jakes anchors) covering the tile into LDS, then every lane
// accumulates R consecutive outputs with a register sliding window over the
// input: one LDS read of x and one broadcast LDS read of the tap pair per tap
// feed R complex multiply-adds.  This is a short time-varying FIR, not a dense
// contraction, so it runs on the vector ALUs (no MFMA).
//
// The per-sample arithmetic is fixed: for every output, taps are formed as
// h = H + a * D (a = integer offset inside the snapshot block or anchor
// interval, D the per-sample increment) and accumulated over t, then l,
// ascending, with explicit fused multiply-adds, so a result does not depend
// on the tile, the batch or the kernel variant that produced it.
#include "tt_internal.h"

namespace tt {

extern __shared__ __align__(16) unsigned char g_lds[];

__device__ __forceinline__ float2 load_iq(const void* x, int fmt, int64_t idx)
{
    if (fmt == IQ_CI16) {
        const short2 v = reinterpret_cast<const short2*>(x)[idx];
        return make_float2((float)v.x * (1.0f / 4096.0f), (float)v.y * (1.0f / 4096.0f));
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

// Encode one output sample; returns the number of clamped components.
__device__ __forceinline__ int store_iq(void* out, int fmt, int64_t idx, float2 v)
{
    if (fmt == IQ_CI16) {
        float a = rintf(v.x * 4096.0f);
        float b = rintf(v.y * 4096.0f);
        int sat = (a > 32767.0f || a < -32768.0f) + (b > 32767.0f || b < -32768.0f);
        a = fminf(fmaxf(a, -32768.0f), 32767.0f);
        b = fminf(fmaxf(b, -32768.0f), 32767.0f);
        reinterpret_cast<short2*>(out)[idx] = make_short2((short)a, (short)b);
        return sat;
    }
    reinterpret_cast<float2*>(out)[idx] = v;
    return 0;
}

__device__ __forceinline__ int64_t floor_div64(int64_t a, int64_t b)
{
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

int lds_bytes_for(int T, int Lp, int n_tx, int n_rx, int nblocks)
{
    const int xs = n_tx * (Lp + T) * 8;
    const int ts = nblocks * n_rx * n_tx * Lp * 16;
    const int an = (nblocks + 1) * n_rx * n_tx * Lp * 8;  // Jakes anchors before differencing
    return xs + ts + an;
}

// Stage one link's taps for blocks kfirst .. kfirst + nblk - 1 as (H, D) pairs.
__device__ void stage_taps(const LinkDev& lk, int64_t kfirst, int nblk, int Lp, float4* ts, float2* anc)
{
    const int n_rx = lk.n_rx, n_tx = lk.n_tx, L = lk.L;
    const int rtl = n_rx * n_tx * Lp;
    if (lk.mode != M_JAKES) {
        const int per = n_rx * n_tx * L;
        const float invP = 1.0f / (float)lk.period;
        for (int e = threadIdx.x; e < nblk * rtl; e += kBlock) {
            const int blk = e / rtl;
            const int q = e - blk * rtl;
            const int l = q % Lp;
            const int rt = q / Lp;  // r * n_tx + t
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (l < L) {
                const int64_t k = kfirst + blk;
                const int64_t s0 = (k % lk.ring_cap) * per + (int64_t)rt * L + l;
                const float2 h = load_tap(lk.ring, lk.tap_fmt, s0);
                v.x = h.x;
                v.y = h.y;
                if (lk.mode == M_LINEAR) {
                    const int64_t s1 = ((k + 1) % lk.ring_cap) * per + (int64_t)rt * L + l;
                    const float2 hn = load_tap(lk.ring, lk.tap_fmt, s1);
                    v.z = (hn.x - h.x) * invP;
                    v.w = (hn.y - h.y) * invP;
                }
            }
            ts[e] = v;
        }
        return;
    }
    // JAKES: exact anchors at n = a K for a = kfirst .. kfirst + nblk, then
    // per-sample increments D = (h_{a+1} - h_a) / K.
    const int K = lk.period;
    for (int e = threadIdx.x; e < (nblk + 1) * rtl; e += kBlock) {
        const int a = e / rtl;
        const int q = e - a * rtl;
        const int l = q % Lp;
        const int rt = q / Lp;
        float2 h = make_float2(0.f, 0.f);
        if (l < L) {
            const double n = (double)((kfirst + a) * (int64_t)K);
            const JakesPair* jp = lk.jakes + ((int64_t)rt * L + l) * kJakesPairs;
#pragma unroll
            for (int m = 0; m < kJakesPairs; ++m) {
                const JakesPair p = jp[m];
                double c = p.nu * n;
                c = c - floor(c);
                float s, co;
                sincospif(2.0f * (float)c, &s, &co);
                h.x = fmaf(co, p.a.x, h.x);
                h.x = fmaf(s, p.b.x, h.x);
                h.y = fmaf(co, p.a.y, h.y);
                h.y = fmaf(s, p.b.y, h.y);
            }
        }
        anc[e] = h;
    }
    __syncthreads();
    const float invK = 1.0f / (float)K;
    for (int e = threadIdx.x; e < nblk * rtl; e += kBlock) {
        const float2 h0 = anc[e];
        const float2 h1 = anc[e + rtl];
        ts[e] = make_float4(h0.x, h0.y, (h1.x - h0.x) * invK, (h1.y - h0.y) * invK);
    }
}

// Accumulate one link into acc[r][q] for the lane's R consecutive outputs.
// xs: staged input, residue-class layout: relative sample index i (from -HP)
// lives at row (i + HP) % R, column (i + HP) / R, rows of S float2, so the R
// lanes' reads of one step are consecutive words.  tp: tap pairs (H, D) of
// the lane's snapshot block, [r][t][l] with l padded to Lp.
template <int R, int NRX, bool INTERP>
__device__ __forceinline__ void fir_link(const float2* __restrict__ xs, const float4* __restrict__ tp, int n_tx,
                                         int Lp, int HP, int S, int tid, float a0, float (&acc)[NRX][R][2])
{
    for (int t = 0; t < n_tx; ++t) {
        const float2* xr = xs + t * R * S;
        float2 w[R];
#pragma unroll
        for (int q = 0; q < R; ++q)
            w[q] = xr[q * S + tid + HP / R];
        const float4* tpt = tp + t * Lp;
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

template <int R, int NRX>
__global__ __launch_bounds__(kBlock) void k_fir(const JobDev* __restrict__ jobs, int njobs,
                                                const LinkDev* __restrict__ links,
                                                const __half2* __restrict__ noise, int64_t npool,
                                                int iq_fmt, unsigned long long* __restrict__ sat)
{
    constexpr int T = kBlock * R;
    const int b = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile0 <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const JobDev& job = jobs[lo];
    const int N = job.N;
    const int tile = b - job.tile0;
    const int i0 = tile * T;
    const int tid = threadIdx.x;
    const int ibase = i0 + tid * R;
    const int tile_len = min(T, N - i0);

    float acc[NRX][R][2];
#pragma unroll
    for (int r = 0; r < NRX; ++r)
#pragma unroll
        for (int q = 0; q < R; ++q)
            acc[r][q][0] = acc[r][q][1] = 0.f;

    for (int li = 0; li < job.nlinks; ++li) {
        const LinkDev& lk = links[job.link0 + li];
        const int L = lk.L, n_tx = lk.n_tx;
        const int Lp = (L + R - 1) / R * R;
        const int HP = Lp;
        const int S = (HP + T) / R;
        float2* xs = reinterpret_cast<float2*>(g_lds);
        const int64_t nfirst = lk.n0 + i0;
        const int P = lk.period;
        const int64_t kfirst = floor_div64(nfirst, P);
        const int64_t klast = floor_div64(nfirst + tile_len - 1, P);
        const int nblk = (int)(klast - kfirst + 1);
        float4* ts = reinterpret_cast<float4*>(g_lds + (size_t)n_tx * (HP + T) * 8);
        float2* anc = reinterpret_cast<float2*>(reinterpret_cast<unsigned char*>(ts) +
                                                (size_t)nblk * NRX * n_tx * Lp * 16);

        // ---- stage input + halo (relative indices -HP .. T-1) ----
        for (int t = 0; t < n_tx; ++t) {
            const int64_t xrow = (int64_t)t * N;
            for (int m = tid; m < HP + T; m += kBlock) {
                const int i = i0 + m - HP;  // slot-relative sample
                float2 v = make_float2(0.f, 0.f);
                if (i >= 0) {
                    if (i < N)
                        v = load_iq(lk.x, iq_fmt, xrow + i);
                } else if (i >= -(L - 1)) {
                    v = lk.hist[t * kHist + (L - 1) + i];
                }
                xs[(t * R + (m % R)) * S + m / R] = v;
            }
        }
        stage_taps(lk, kfirst, nblk, Lp, ts, anc);
        __syncthreads();

        // ---- history rewrite (first tile): last L-1 inputs of this call ----
        if (i0 == 0 && lk.write_hist && L > 1) {
            for (int e = tid; e < n_tx * (L - 1); e += kBlock) {
                const int t = e / (L - 1);
                const int k = e - t * (L - 1);
                const int s = N - (L - 1) + k;
                float2 v;
                if (s >= 0) {
                    v = load_iq(lk.x, iq_fmt, (int64_t)t * N + s);
                } else {
                    const int m = s + HP;  // staged from the old history
                    v = xs[(t * R + (m % R)) * S + m / R];
                }
                lk.hist[t * kHist + k] = v;
            }
        }

        // ---- FIR ----
        if (ibase < N) {
            const int rem0 = (int)(nfirst - kfirst * P);
            const int rem = rem0 + tid * R;
            const int blk = rem / P;
            const float a0 = (float)(rem - blk * P);
            const float4* tp = ts + (size_t)blk * NRX * n_tx * Lp;
            if (lk.mode != M_HOLD)
                fir_link<R, NRX, true>(xs, tp, n_tx, Lp, HP, S, tid, a0, acc);
            else
                fir_link<R, NRX, false>(xs, tp, n_tx, Lp, HP, S, tid, a0, acc);
        }
        __syncthreads();  // LDS is restaged for the next link
    }

    // ---- epilogue ----
    if (ibase >= N)
        return;
    int nsat = 0;
    if (job.kind == J_FINAL) {
#pragma unroll
        for (int r = 0; r < NRX; ++r) {
            int64_t p = (job.noise_off[r] + job.noise_n0 + ibase) % npool;
            if (p < 0)
                p += npool;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int i = ibase + q;
                if (i < N) {
                    const float2 wv = __half22float2(noise[p]);
                    float2 v;
                    v.x = fmaf(job.sigma, wv.x, acc[r][q][0]);
                    v.y = fmaf(job.sigma, wv.y, acc[r][q][1]);
                    nsat += store_iq(job.out, iq_fmt, (int64_t)r * N + i, v);
                }
                if (++p == npool)
                    p = 0;
            }
        }
    } else {
        float2* out = reinterpret_cast<float2*>(job.out);
#pragma unroll
        for (int r = 0; r < NRX; ++r)
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int i = ibase + q;
                if (i < N)
                    out[(int64_t)r * N + i] = make_float2(acc[r][q][0], acc[r][q][1]);
            }
    }
    if (nsat)
        atomicAdd(sat, (unsigned long long)nsat);
}

template <int R, int NRX>
static hipError_t launch_fir_t(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                               const __half2* noise, int64_t npool, int iq_fmt, unsigned long long* sat,
                               hipStream_t st)
{
    hipLaunchKernelGGL((k_fir<R, NRX>), dim3(s.total_tiles), dim3(kBlock), s.lds_bytes, st, jobs, njobs,
                       links, noise, npool, iq_fmt, sat);
    return hipGetLastError();
}

template <int R>
static hipError_t launch_fir_r(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                               const __half2* noise, int64_t npool, int iq_fmt, unsigned long long* sat,
                               hipStream_t st)
{
    switch (s.nrx) {
    case 1: return launch_fir_t<R, 1>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    case 2: return launch_fir_t<R, 2>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    case 3: return launch_fir_t<R, 3>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    case 4: return launch_fir_t<R, 4>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fir(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                      const __half2* noise, int64_t npool, int iq_fmt, unsigned long long* sat,
                      hipStream_t st)
{
    if (s.total_tiles <= 0)
        return hipSuccess;
    switch (s.R) {
    case 1: return launch_fir_r<1>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    case 2: return launch_fir_r<2>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    case 4: return launch_fir_r<4>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    case 8: return launch_fir_r<8>(s, jobs, njobs, links, noise, npool, iq_fmt, sat, st);
    }
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// UL second pass: fixed-order sum over groups, cell noise, encode.
// grid: (ceil(max_n / 256), max_ant, nred)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_reduce(const ReduceDev* __restrict__ reds,
                                                   const __half2* __restrict__ noise, int64_t npool,
                                                   int iq_fmt, unsigned long long* __restrict__ sat)
{
    const ReduceDev& rd = reds[blockIdx.z];
    const int r = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (r >= rd.n_ant || i >= rd.N)
        return;
    float2 v = make_float2(0.f, 0.f);
    if (!(rd.flags & 1))
        v = rd.acc[(int64_t)r * rd.stride + i];
    const int64_t gstride = (int64_t)rd.n_ant * rd.N;
    for (int g = 0; g < rd.ngroups; ++g) {
        const float2 p = rd.partial[g * gstride + (int64_t)r * rd.N + i];
        v.x += p.x;
        v.y += p.y;
    }
    if (rd.flags & 2) {
        int64_t p = (rd.noise_off[r] + rd.m0 + i) % npool;
        if (p < 0)
            p += npool;
        const float2 wv = __half22float2(noise[p]);
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
                         int64_t npool, int iq_fmt, unsigned long long* sat, hipStream_t st)
{
    if (nred <= 0 || max_n <= 0)
        return hipSuccess;
    dim3 grid((max_n + kBlock - 1) / kBlock, max_ant, nred);
    hipLaunchKernelGGL(k_reduce, grid, dim3(kBlock), 0, st, red, noise, npool, iq_fmt, sat);
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
