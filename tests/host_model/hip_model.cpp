// CPU model of the HIP runtime calls and kernel launches the library's host
// code makes, for running that host code (arena, admission, descriptor
// building, serving loop, host IQ pipeline) under AddressSanitizer and
// UndefinedBehaviorSanitizer on a machine without a GPU.  Test
// infrastructure only: it is linked into the sanitizer driver, never into
// the library.
//
// Device memory is host memory.  Copies and fills run at once; events and
// streams complete at once; graph capture records nothing (the launches made
// while capturing are checked when they are made).  Each kernel launch is
// replaced by a checker that reads every descriptor it is given (so an
// overrun of a descriptor table is an ASan report) and verifies that every
// span the kernel would touch lies inside one live allocation, with the
// launch shape the kernel assumes.  A violation prints the launch and aborts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "tt_internal.h"

namespace {

std::mutex g_mu;
std::map<uintptr_t, size_t> g_blocks;  // live allocations: start -> bytes
int64_t g_launches = 0;

[[noreturn]] void die(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "hip_model: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
    std::abort();
}

void* take(size_t bytes)
{
    const size_t n = (bytes + 255) / 256 * 256;
    void* p = std::aligned_alloc(256, n ? n : 256);
    if (!p)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    g_blocks[(uintptr_t)p] = bytes;
    return p;
}

void give(void* p)
{
    if (!p)
        return;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_blocks.find((uintptr_t)p);
        if (it == g_blocks.end())
            die("free of %p, which is not a live allocation", p);
        g_blocks.erase(it);
    }
    std::free(p);
}

// [p, p + bytes) inside one live allocation
void span(const void* p, int64_t bytes, const char* what)
{
    if (bytes < 0)
        die("%s: negative extent %lld", what, (long long)bytes);
    if (bytes == 0)
        return;
    if (!p)
        die("%s: null pointer for %lld bytes", what, (long long)bytes);
    std::lock_guard<std::mutex> lk(g_mu);
    const uintptr_t a = (uintptr_t)p;
    auto it = g_blocks.upper_bound(a);
    if (it == g_blocks.begin())
        die("%s: %p is not inside an allocation", what, p);
    --it;
    if (a + (uintptr_t)bytes > it->first + it->second)
        die("%s: [%p, +%lld) runs past its allocation [%p, +%zu)", what, p, (long long)bytes, (void*)it->first,
            it->second);
}

struct Opaque {
    int tag;
};
template <class T>
T make_handle()
{
    return reinterpret_cast<T>(new Opaque{1});
}
template <class T>
void drop_handle(T h)
{
    delete reinterpret_cast<Opaque*>(h);
}

}  // namespace

// --------------------------------------------------------------------------
// runtime calls
// --------------------------------------------------------------------------
extern "C" {

hipError_t hipMalloc(void** p, size_t bytes)
{
    *p = take(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p)
{
    give(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int)
{
    *p = take(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p)
{
    give(p);
    return hipSuccess;
}
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned int)
{
    span(h, 1, "hipHostGetDevicePointer");
    *d = h;
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind)
{
    std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t)
{
    std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemset(void* dst, int v, size_t bytes)
{
    span(dst, (int64_t)bytes, "hipMemset");
    std::memset(dst, v, bytes);
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int)
{
    *v = 256;
    return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "modelled HIP error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int)
{
    *s = make_handle<hipStream_t>();
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    drop_handle(s);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }

hipError_t hipEventCreate(hipEvent_t* e)
{
    *e = make_handle<hipEvent_t>();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int)
{
    *e = make_handle<hipEvent_t>();
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    drop_handle(e);
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    return e ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t)
{
    *ms = 0.001f;
    return hipSuccess;
}

hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g)
{
    *g = make_handle<hipGraph_t>();
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t, hipGraphNode_t*, char*, size_t)
{
    *x = make_handle<hipGraphExec_t>();
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g)
{
    drop_handle(g);
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x)
{
    drop_handle(x);
    return hipSuccess;
}

}  // extern "C"

// --------------------------------------------------------------------------
// kernel launches: checkers
// --------------------------------------------------------------------------
namespace tt {

namespace {
int sample_bytes(int iq_fmt) { return iq_fmt == IQ_CI16 ? 4 : 8; }
int tap_bytes(int tap_fmt) { return tap_fmt == TAP_F16 ? 4 : 8; }
int64_t fdiv(int64_t a, int64_t b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// The snapshots (or selected pairs) one link's convolution reads for a call of N samples.
void check_link(const LinkDev& lk, int N, int iq_fmt, int nrx, int kind, const char* what)
{
    if (lk.n_rx != nrx)
        die("%s: link with %d receive antennas in a launch of %d", what, lk.n_rx, nrx);
    if (lk.n_tx < 1 || lk.n_tx > kMaxAnt || lk.L < 1 || lk.L > kMaxTaps || lk.period < 1)
        die("%s: link shape n_tx %d L %d period %d", what, lk.n_tx, lk.L, lk.period);
    if (lk.mode != M_HOLD && lk.mode != M_LINEAR)
        die("%s: convolution link mode %d", what, lk.mode);
    if (lk.r0 < 0 || lk.r0 >= lk.period)
        die("%s: r0 %d outside the block of period %d", what, lk.r0, lk.period);
    span(lk.x, (int64_t)lk.n_tx * N * sample_bytes(iq_fmt), "link input");
    span(lk.hist, (int64_t)lk.n_tx * kHist * 8, "link history");
    const int64_t per = (int64_t)lk.n_rx * lk.n_tx * lk.L;
    const int64_t nblk = (lk.r0 + (int64_t)N - 1) / lk.period + 1;
    if (lk.nsel > 0) {
        if (lk.nsel > lk.L)
            die("%s: %d selected of %d taps", what, lk.nsel, lk.L);
        const int64_t groups = (lk.k0 + nblk - lk.sk0) * lk.n_rx * lk.n_tx;
        span(lk.spairs, groups * lk.nsel * 16, "sparse pairs");
        span(lk.sdelay, groups * lk.nsel * 4, "sparse delays");
    } else if (lk.ring_cap > 0) {
        if (lk.slot0 < 0 || lk.slot0 >= lk.ring_cap)
            die("%s: ring slot %d of %d", what, lk.slot0, lk.ring_cap);
        span(lk.ring, lk.ring_cap * per * tap_bytes(lk.tap_fmt), "tap ring");
    } else {
        const int64_t last = lk.k0 + nblk - 1 + (lk.mode == M_LINEAR ? 1 : 0);
        if (lk.k0 < lk.kbase)
            die("%s: first snapshot %lld before the buffer's %lld", what, (long long)lk.k0, (long long)lk.kbase);
        span(lk.ring, (last - lk.kbase + 1) * per * tap_bytes(lk.tap_fmt), "caller snapshots / anchors");
    }
    if (kind == J_DL)
        span(lk.y, (int64_t)lk.n_rx * N * sample_bytes(iq_fmt), "DL output");
}

void check_reduce(const ReduceDev& r, int iq_fmt, const char* what)
{
    if (r.n_ant < 1 || r.n_ant > kMaxAnt || r.N < 0 || r.N > r.stride || r.ngroups < 0)
        die("%s: reduction n_ant %d N %d stride %d groups %d", what, r.n_ant, r.N, r.stride, r.ngroups);
    span(r.partial, (int64_t)r.ngroups * r.n_ant * r.N * 8, "UL partials");
    span(r.acc, (int64_t)r.n_ant * r.stride * 8, "UL accumulator");
    if (r.flags & 2)
        span(r.z, (int64_t)r.n_ant * r.N * sample_bytes(iq_fmt), "UL output");
    if (r.counters)
        span(r.counters, ((int64_t)r.N + kBlock - 1) / kBlock * 4, "UL tile counters");
}
}  // namespace

hipError_t launch_fir(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                      const ReduceDev* reds, const __half2* noise, int32_t npool, int iq_fmt,
                      unsigned long long* sat, hipStream_t, hipEvent_t, hipEvent_t)
{
    ++g_launches;
    if (s.R != 1 && s.R != 2 && s.R != 4 && s.R != 8)
        die("k_fir: R %d", s.R);
    if (s.nrx < 1 || s.nrx > kMaxAnt || s.lds_bytes <= 0 || s.lds_bytes > 64 * 1024)
        die("k_fir: nrx %d lds %d", s.nrx, s.lds_bytes);
    if (s.grid < 1 || s.grid > s.total_tiles)
        die("k_fir: grid %d for %d tiles", s.grid, s.total_tiles);
    if (s.rawx_bytes + s.rawt_bytes > 0 && s.raw_off + s.rawx_bytes + s.rawt_bytes > s.lds_bytes)
        die("k_fir: prefetch area past the LDS size");
    span(noise, (int64_t)npool * 4, "noise pool");
    span(sat, 8, "saturation counter");
    int tiles = 0, uniform = -1;
    for (int j = 0; j < njobs; ++j) {
        const JobDev& jb = jobs[j];
        if (jb.sub != 1 && (jb.kind != J_DL || (jb.sub != 2 && jb.sub != 4)))
            die("k_fir: job %d kind %d with %d lane tiles per item", j, jb.kind, jb.sub);
        const int T = kBlock * s.R * jb.sub;
        if (jb.tile0 != tiles || jb.ntiles != (jb.N + T - 1) / T || jb.N < 1)
            die("k_fir: job %d tile0 %d ntiles %d N %d (expected tile0 %d)", j, jb.tile0, jb.ntiles, jb.N, tiles);
        // the staging the kernel lays out for the job's items fits the LDS
        // (before the prefetch area when there is one)
        const int room = s.rawx_bytes + s.rawt_bytes > 0 ? s.raw_off : s.lds_bytes;
        for (int i = 0; i < jb.nlinks; ++i) {
            const LinkDev& lk = links[jb.link0 + i];
            if (lk.period < 1 || lk.n_tx < 1 || lk.n_rx < 1)
                continue;  // check_link reports it
            const int Lp = (lk.L + s.R - 1) / s.R * s.R;
            const int HP = (Lp + 3) / 4 * 4;
            const int Srow = (HP + T) / s.R | 1;
            const int xs = lk.n_tx * s.R * Srow * 8;
            for (int t = 0; t < jb.ntiles; ++t) {
                const int i0 = t * T;
                const int len = std::min(T, jb.N - i0);
                const int rem0 = (int)((lk.r0 + (int64_t)i0) % lk.period);
                const int nblk = (rem0 + len - 1) / lk.period + 1;
                const int ne = nblk * lk.n_rx * lk.n_tx * Lp;
                int need = xs + ne * 16;
                if (lk.nsel > 0)
                    need += ((ne * 12 + 15) & ~15) + nblk * lk.n_rx * lk.n_tx * lk.nsel * (16 + 4 * s.R);
                if (need > room)
                    die("k_fir: job %d link %d tile %d stages %d bytes of LDS, %d available", j, i, t, need, room);
            }
        }
        uniform = uniform == -1 ? jb.ntiles : (uniform == jb.ntiles ? uniform : 0);
        tiles += jb.ntiles;
        if (jb.nlinks < 1 || jb.link0 < 0)
            die("k_fir: job %d links %d..+%d", j, jb.link0, jb.nlinks);
        if (jb.kind != J_DL && jb.kind != J_FINAL && jb.kind != J_PARTIAL)
            die("k_fir: job kind %d", jb.kind);
        for (int i = 0; i < jb.nlinks; ++i)
            check_link(links[jb.link0 + i], jb.N, iq_fmt, s.nrx, jb.kind, "k_fir");
        if (jb.kind == J_FINAL)
            span(jb.out, (int64_t)jb.n_out * jb.N * sample_bytes(iq_fmt), "UL output");
        if (jb.kind == J_PARTIAL)
            span(jb.out, (int64_t)jb.n_out * jb.N * 8, "UL partial");
        if (jb.kind == J_PARTIAL && jb.red >= 0)
            check_reduce(reds[jb.red], iq_fmt, "k_fir fused reduction");
        if (jb.kind != J_DL && jb.n_out != s.nrx)
            die("k_fir: UL job with %d outputs in a launch of %d", jb.n_out, s.nrx);
    }
    if (tiles != s.total_tiles)
        die("k_fir: %d tiles in the jobs, %d in the shape", tiles, s.total_tiles);
    bool multi = false;
    for (int j = 0; j < njobs; ++j)
        multi = multi || jobs[j].sub > 1;
    if (s.subtiles != (multi ? 1 : 0))
        die("k_fir: subtiles flag %d with%s multi-tile jobs", s.subtiles, multi ? "" : "out");
    if (s.tiles_per_job > 0 && s.tiles_per_job != uniform)
        die("k_fir: tiles_per_job %d but jobs are not uniform", s.tiles_per_job);
    return hipSuccess;
}

hipError_t launch_anchor(const AnchorDev* ent, int n, int blocks, hipStream_t, hipEvent_t, hipEvent_t)
{
    ++g_launches;
    int b = 0;
    for (int i = 0; i < n; ++i) {
        const AnchorDev& e = ent[i];
        if (e.block0 != b || e.k0 < 0 || e.count < 1 || e.per < 1 || e.K < 1)
            die("k_anchor: entry %d block0 %d (expected %d) k0 %lld count %d", i, e.block0, b, (long long)e.k0,
                e.count);
        span(e.jakes, (int64_t)e.per * kJakesPairs * kJakesPairBytes, "Jakes parameters");
        span(e.out, (int64_t)e.count * e.per * 8, "anchor table");
        const int64_t ngrp = (e.k0 + e.count - 1) / kAnchorGroup - e.k0 / kAnchorGroup + 1;
        b += (int)((ngrp * e.per + kBlock - 1) / kBlock);
    }
    if (b != blocks)
        die("k_anchor: %d workgroups launched, entries need %d", blocks, b);
    return hipSuccess;
}

hipError_t launch_select(const SelectDev* ent, int n, int blocks, hipStream_t)
{
    ++g_launches;
    for (int i = 0; i < n; ++i) {
        const SelectDev& e = ent[i];
        const int64_t per = (int64_t)e.n_rx * e.n_tx * e.L;
        const int64_t groups = (int64_t)e.nblk * e.n_rx * e.n_tx;
        const int gl = e.L <= 8 ? 8 : e.L <= 16 ? 16 : e.L <= 32 ? 32 : 64;
        if ((groups * gl + kSelRounds * kBlock - 1) / (kSelRounds * kBlock) > blocks)
            die("k_select: entry %d needs more than %d workgroups", i, blocks);
        const int64_t snaps = e.nblk + (e.mode == M_LINEAR ? 1 : 0);
        if (e.ring_cap > 0)
            span(e.ring, e.ring_cap * per * tap_bytes(e.tap_fmt), "selection ring");
        else
            span(e.ring, (e.s0 + snaps) * per * tap_bytes(e.tap_fmt), "selection snapshots");
        span(e.pairs, groups * e.nsel * 16, "selection pairs");
        span(e.delay, groups * e.nsel * 4, "selection delays");
    }
    return hipSuccess;
}

hipError_t launch_reduce(const ReduceDev* red, int nred, int max_n, int max_ant, const __half2* noise,
                         int32_t npool, int iq_fmt, unsigned long long* sat, hipStream_t)
{
    ++g_launches;
    span(noise, (int64_t)npool * 4, "noise pool");
    span(sat, 8, "saturation counter");
    for (int i = 0; i < nred; ++i) {
        if (red[i].N > max_n || red[i].n_ant > max_ant)
            die("k_reduce: entry %d beyond the launch bounds", i);
        check_reduce(red[i], iq_fmt, "k_reduce");
    }
    return hipSuccess;
}

hipError_t launch_ingest(const IngestDev* ent, int n, int64_t max_taps, hipStream_t)
{
    ++g_launches;
    for (int i = 0; i < n; ++i) {
        const IngestDev& e = ent[i];
        if (e.count > e.cap || e.count < 0 || (int64_t)e.count * e.per > max_taps)
            die("k_ingest: entry %d count %d cap %d", i, e.count, e.cap);
        span(e.src, (int64_t)e.count * e.per * e.bytes_per_tap, "ingest source");
        span(e.ring, (int64_t)e.cap * e.per * e.bytes_per_tap, "ingest ring");
    }
    return hipSuccess;
}

hipError_t launch_resample(const ResampleDev* ent, int n, int max_count, hipStream_t)
{
    ++g_launches;
    for (int i = 0; i < n; ++i) {
        const ResampleDev& e = ent[i];
        if (e.count > max_count || e.count > e.cap)
            die("k_resample: entry %d count %d", i, e.count);
        span(e.delay, (int64_t)e.count * e.n_paths * 8, "CIR delays");
        span(e.gain, (int64_t)e.count * e.n_paths * e.n_rx * e.n_tx * 8, "CIR gains");
        span(e.ring, (int64_t)e.cap * e.n_rx * e.n_tx * e.L * tap_bytes(e.tap_fmt), "CIR ring");
    }
    return hipSuccess;
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t)
{
    ++g_launches;
    span(p, bytes, "k_zero");
    std::memset(p, 0, (size_t)bytes);
    return hipSuccess;
}

hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t)
{
    ++g_launches;
    span(dst, bytes, "k_copy destination");
    span(src, bytes, "k_copy source");
    std::memmove(dst, src, (size_t)bytes);
    return hipSuccess;
}

unsigned char* g_scratch = nullptr;
hipError_t noalloc_scratch_init(int)
{
    if (!g_scratch)
        g_scratch = static_cast<unsigned char*>(take(kNoallocScratchBytes));
    return g_scratch ? hipSuccess : hipErrorOutOfMemory;
}
void* noalloc_scratch(int) { return g_scratch; }

}  // namespace tt

extern "C" int64_t hip_model_launches(void) { return g_launches; }
// live allocations apart from the allocation-free call's scratch (a static
// device array in the library, held until the process ends)
extern "C" int64_t hip_model_live_blocks(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (int64_t)g_blocks.size() - (tt::g_scratch ? 1 : 0);
}
