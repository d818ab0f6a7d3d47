// Host IQ coupling: the UEs and the gNB of the paper exchange IQ with the
// channel through host memory (rfsim's socket transport, Sec. III-A).  Here a
// producer writes each slot's IQ into pinned host buffers; one H2D copy per
// slot moves it to HBM on a copy stream, the slot runs on the channel's
// stream, and one D2H copy on a second copy stream returns the outputs.
// `depth` slot buffers rotate, so the copies of neighbouring slots overlap
// the kernels of the current one (PCIe is full duplex).
#include "tt_internal.h"
#include "tt_channel.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

tt_status io_fail(tt_status s, const char* m)
{
    tt::set_error(m);
    return s;
}

struct Buf {
    char* h_in = nullptr;      // pinned
    char* h_out = nullptr;     // pinned
    char* d_in = nullptr;
    char* d_out = nullptr;
    hipEvent_t ev_in = nullptr, ev_slot = nullptr, ev_out = nullptr;
    bool busy = false;         // submitted, completion not yet observed
    Clock::time_point t_sub{};
    double lat_us = -1.0;      // submit -> outputs observed in host memory
};

}  // namespace

struct tt_io {
    tt_channel* ch = nullptr;
    int device = 0;
    int32_t cell = 0, n = 0, N = 0, n_ant = 1;
    int64_t sb = 4;
    std::vector<int32_t> ue, n_tx, n_rx;
    int64_t in_bytes = 0, out_bytes = 0;
    hipStream_t s_h2d = nullptr, s_d2h = nullptr;
    std::vector<Buf> bufs;
    // per-buffer slot descriptions handed to tt_channel_apply_slot
    std::vector<std::vector<const void*>> dl_x, ul_x;
    std::vector<std::vector<void*>> dl_y, ul_z;
    std::vector<int32_t> cell_samples;

    tt_status observe(Buf& b, bool block)
    {
        if (!b.busy)
            return TT_OK;
        hipError_t e = block ? hipEventSynchronize(b.ev_out) : hipEventQuery(b.ev_out);
        if (e == hipErrorNotReady)
            return TT_OK;
        const Clock::time_point now = Clock::now();
        b.busy = false;
        b.lat_us = std::chrono::duration<double, std::micro>(now - b.t_sub).count();
        if (e != hipSuccess)
            return io_fail(TT_E_DEVICE, "tt_io: device error while waiting for a slot");
        return TT_OK;
    }

    void release()
    {
        for (Buf& b : bufs) {
            if (b.busy)
                (void)hipEventSynchronize(b.ev_out);
            if (b.h_in)
                (void)hipHostFree(b.h_in);
            if (b.h_out)
                (void)hipHostFree(b.h_out);
            if (b.d_in)
                (void)hipFree(b.d_in);
            if (b.d_out)
                (void)hipFree(b.d_out);
            for (hipEvent_t ev : {b.ev_in, b.ev_slot, b.ev_out})
                if (ev)
                    (void)hipEventDestroy(ev);
        }
        bufs.clear();
        if (s_h2d)
            (void)hipStreamDestroy(s_h2d);
        if (s_d2h)
            (void)hipStreamDestroy(s_d2h);
        s_h2d = s_d2h = nullptr;
    }
};

extern "C" {

tt_status tt_io_create(tt_channel* ch, const tt_io_cfg* cfg, tt_io** out)
{
    if (!ch || !cfg || !out)
        return io_fail(TT_E_INVALID, "tt_io_create: null argument");
    *out = nullptr;
    int n_cells = 0;
    const tt_cell_cfg* cells = tt::channel_cells(ch, &n_cells);
    if (cfg->cell < 0 || cfg->cell >= n_cells)
        return io_fail(TT_E_INVALID, "tt_io_create: unknown cell");
    if (cfg->n_ues < 1 || !cfg->ue)
        return io_fail(TT_E_INVALID, "tt_io_create: n_ues must be >= 1 with a UE list");
    if (cfg->n_samples < 1 || cfg->n_samples > cells[cfg->cell].max_samples)
        return io_fail(TT_E_INVALID, "tt_io_create: n_samples must be 1..the cell's max_samples");
    if (cfg->depth < 1 || cfg->depth > TT_IO_MAX_DEPTH)
        return io_fail(TT_E_INVALID, "tt_io_create: depth out of range");
    std::vector<char> seen;
    tt_io* io = new tt_io();
    io->ch = ch;
    io->device = tt::channel_device(ch);
    io->cell = cfg->cell;
    io->n = cfg->n_ues;
    io->N = cfg->n_samples;
    io->n_ant = cells[cfg->cell].n_ant;
    io->sb = tt::channel_iq_fmt(ch) == tt::IQ_CI16 ? 4 : 8;
    for (int i = 0; i < cfg->n_ues; ++i) {
        const int u = cfg->ue[i];
        const tt_ue_cfg* c = tt::channel_ue(ch, u);
        if (!c) {
            delete io;
            return io_fail(TT_E_INVALID, "tt_io_create: unknown UE");
        }
        if (c->cell != cfg->cell || c->dl_tx_streams != 0) {
            delete io;
            return io_fail(TT_E_INVALID, "tt_io_create: every UE must be served by the cell's own DL stream");
        }
        if ((int)seen.size() <= u)
            seen.resize(u + 1, 0);
        if (seen[u]) {
            delete io;
            return io_fail(TT_E_INVALID, "tt_io_create: UE listed twice");
        }
        seen[u] = 1;
        io->ue.push_back(u);
        io->n_tx.push_back(c->n_tx);
        io->n_rx.push_back(c->n_rx);
    }
    const int64_t N = io->N, sb = io->sb;
    int64_t in_samples = (int64_t)io->n_ant * N, out_samples = 0;
    for (int i = 0; i < io->n; ++i) {
        in_samples += (int64_t)io->n_tx[i] * N;
        out_samples += (int64_t)io->n_rx[i] * N;
    }
    out_samples += (int64_t)io->n_ant * N;
    io->in_bytes = in_samples * sb;
    io->out_bytes = out_samples * sb;
    hipError_t e = hipSetDevice(io->device);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&io->s_h2d, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&io->s_d2h, hipStreamNonBlocking);
    io->bufs.resize(cfg->depth);
    for (int b = 0; b < cfg->depth && e == hipSuccess; ++b) {
        Buf& B = io->bufs[b];
        e = hipHostMalloc((void**)&B.h_in, io->in_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&B.h_out, io->out_bytes, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipMalloc((void**)&B.d_in, io->in_bytes);
        if (e == hipSuccess)
            e = hipMalloc((void**)&B.d_out, io->out_bytes);
        for (hipEvent_t* ev : {&B.ev_in, &B.ev_slot, &B.ev_out})
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        io->release();
        delete io;
        return io_fail(TT_E_NOMEM, "tt_io_create: allocation of the slot buffers failed");
    }
    // slot descriptions: in = [gNB DL: n_ant][N] then per UE [n_tx][N];
    // out = per UE [n_rx][N] then the cell's UL [n_ant][N]
    io->dl_x.resize(cfg->depth);
    io->ul_x.resize(cfg->depth);
    io->dl_y.resize(cfg->depth);
    io->ul_z.assign(cfg->depth, std::vector<void*>(n_cells, nullptr));
    io->cell_samples.assign(n_cells, 0);
    io->cell_samples[io->cell] = io->N;
    for (int b = 0; b < cfg->depth; ++b) {
        const Buf& B = io->bufs[b];
        int64_t off = (int64_t)io->n_ant * N * sb;
        int64_t off_o = 0;
        for (int i = 0; i < io->n; ++i) {
            io->dl_x[b].push_back(B.d_in);
            io->ul_x[b].push_back(B.d_in + off);
            off += (int64_t)io->n_tx[i] * N * sb;
            io->dl_y[b].push_back(B.d_out + off_o);
            off_o += (int64_t)io->n_rx[i] * N * sb;
        }
        io->ul_z[b][io->cell] = B.d_out + off_o;
    }
    *out = io;
    return TT_OK;
}

tt_status tt_io_buffers(tt_io* io, int32_t b, void** in, int64_t* in_bytes, void** out, int64_t* out_bytes)
{
    if (!io || b < 0 || b >= (int)io->bufs.size())
        return io_fail(TT_E_INVALID, "tt_io_buffers: bad buffer index");
    if (in)
        *in = io->bufs[b].h_in;
    if (in_bytes)
        *in_bytes = io->in_bytes;
    if (out)
        *out = io->bufs[b].h_out;
    if (out_bytes)
        *out_bytes = io->out_bytes;
    return TT_OK;
}

tt_status tt_io_submit(tt_io* io, int32_t b)
{
    if (!io || b < 0 || b >= (int)io->bufs.size())
        return io_fail(TT_E_INVALID, "tt_io_submit: bad buffer index");
    Buf& B = io->bufs[b];
    tt_status s = io->observe(B, false);
    if (s != TT_OK)
        return s;
    if (B.busy)
        return io_fail(TT_E_STATE, "tt_io_submit: buffer still in flight (wait for it first)");
    hipError_t e = hipSetDevice(io->device);
    hipStream_t cs = tt::channel_stream(io->ch);
    B.t_sub = Clock::now();
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.d_in, B.h_in, io->in_bytes, hipMemcpyHostToDevice, io->s_h2d);
    if (e == hipSuccess)
        e = hipEventRecord(B.ev_in, io->s_h2d);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(cs, B.ev_in, 0);
    if (e != hipSuccess)
        return io_fail(TT_E_DEVICE, "tt_io_submit: input copy");
    tt_slot sl{};
    sl.n_dl = io->n;
    sl.dl_ue = io->ue.data();
    sl.dl_x = io->dl_x[b].data();
    sl.dl_y = io->dl_y[b].data();
    sl.n_ul = io->n;
    sl.ul_ue = io->ue.data();
    sl.ul_x = io->ul_x[b].data();
    sl.ul_z = io->ul_z[b].data();
    sl.cell_samples = io->cell_samples.data();
    s = tt_channel_apply_slot(io->ch, &sl);
    if (s != TT_OK) {
        // the input copy is queued; keep the buffer busy until it has landed
        (void)hipEventRecord(B.ev_out, io->s_h2d);
        B.busy = true;
        return s;
    }
    e = hipEventRecord(B.ev_slot, cs);
    if (e == hipSuccess)
        e = hipStreamWaitEvent(io->s_d2h, B.ev_slot, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B.h_out, B.d_out, io->out_bytes, hipMemcpyDeviceToHost, io->s_d2h);
    if (e == hipSuccess)
        e = hipEventRecord(B.ev_out, io->s_d2h);
    if (e != hipSuccess)
        return io_fail(TT_E_DEVICE, "tt_io_submit: output copy");
    B.busy = true;
    B.lat_us = -1.0;
    return TT_OK;
}

tt_status tt_io_poll(tt_io* io, int32_t* in_flight)
{
    if (!io)
        return io_fail(TT_E_INVALID, "tt_io_poll: null handle");
    int busy = 0;
    for (Buf& B : io->bufs) {
        tt_status s = io->observe(B, false);
        if (s != TT_OK)
            return s;
        busy += B.busy ? 1 : 0;
    }
    if (in_flight)
        *in_flight = busy;
    return TT_OK;
}

tt_status tt_io_wait(tt_io* io, int32_t b, double* latency_us)
{
    if (!io || b < 0 || b >= (int)io->bufs.size())
        return io_fail(TT_E_INVALID, "tt_io_wait: bad buffer index");
    // observe older completions first so their times are not taken late
    for (Buf& B : io->bufs) {
        tt_status s = io->observe(B, false);
        if (s != TT_OK)
            return s;
    }
    tt_status s = io->observe(io->bufs[b], true);
    if (latency_us)
        *latency_us = io->bufs[b].lat_us;
    return s;
}

tt_status tt_io_destroy(tt_io* io)
{
    if (!io)
        return TT_OK;
    (void)hipSetDevice(io->device);
    io->release();
    delete io;
    return TT_OK;
}

}  // extern "C"
