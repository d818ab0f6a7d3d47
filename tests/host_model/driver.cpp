// Drives the library's host runtime through its C ABI on the CPU model of
// the HIP runtime (hip_model.cpp), built with AddressSanitizer and
// UndefinedBehaviorSanitizer: channel create/destroy, admission and release
// in the arena, tap windows, Jakes anchor tables, every apply entry point
// (including the prepared and allocation-free forms) under a range of launch
// schedules, refusals, the serving loop and the host IQ pipeline.  The model
// checks every kernel launch's descriptors and spans; this program checks the
// status codes and that every allocation is returned at the end.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include <hip/hip_runtime.h>

#include "tt_channel.h"

extern "C" int64_t hip_model_launches(void);
extern "C" int64_t hip_model_live_blocks(void);

namespace {

int g_fail = 0;

void expect(bool ok, const char* what, int line)
{
    if (!ok) {
        std::fprintf(stderr, "driver: line %d: %s (%s)\n", line, what, tt_last_error());
        ++g_fail;
    }
}
#define OK(call) expect((call) == TT_OK, #call, __LINE__)
#define REFUSED(call, code) expect((call) == (code), #call " refused", __LINE__)

void* dev(size_t bytes)
{
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        std::fprintf(stderr, "driver: hipMalloc(%zu)\n", bytes);
        std::exit(2);
    }
    std::memset(p, 0, bytes);
    return p;
}

struct Ue {
    tt_ue_cfg cfg;
    int id = -1;
    int dl_tx = 1, ul_rx = 1;
    std::vector<float> snaps[2];  // host snapshots per direction (f32 complex or f16 pairs as raw bytes)
};

constexpr int kCells = 2;
const double kRate[kCells] = {61.44e6, 122.88e6};
const int kAnt[kCells] = {1, 2};
const int kMax[kCells] = {4096, 8192};
const int64_t kTotal[kCells] = {70000, 120000};  // samples a run takes per cell, at most

std::vector<Ue> make_ues()
{
    std::vector<Ue> v;
    auto add = [&](int cell, int L, int n_tx, int n_rx, int mode, int P, int fmt, int sparse, int dl_streams) {
        Ue u;
        std::memset(&u.cfg, 0, sizeof(u.cfg));
        u.cfg.cell = cell;
        u.cfg.n_taps = L;
        u.cfg.n_tx = n_tx;
        u.cfg.n_rx = n_rx;
        u.cfg.mode = mode;
        u.cfg.snapshot_period = P;
        u.cfg.tap_fmt = fmt;
        // a ring that holds every snapshot of a run
        u.cfg.ring_snapshots = mode == TT_TAPS_JAKES ? 0 : (int32_t)(kTotal[cell] / P + 8);
        u.cfg.dl_sigma = 0.01f;
        u.cfg.sparse_taps = sparse;
        u.cfg.dl_tx_streams = dl_streams;
        for (int a = 0; a < TT_MAX_ANT; ++a)
            u.cfg.dl_noise_off[a] = 17 * (int)v.size() + a;
        u.dl_tx = dl_streams > 0 ? dl_streams : kAnt[cell];
        u.ul_rx = kAnt[cell];
        v.push_back(u);
    };
    add(0, 8, 1, 1, TT_TAPS_HOLD, 128, TT_TAP_F32, 0, 0);
    add(0, 16, 1, 1, TT_TAPS_LINEAR, 64, TT_TAP_F16, 0, 0);
    add(0, 16, 1, 1, TT_TAPS_LINEAR, 100, TT_TAP_F32, 4, 0);   // sparse top-4, odd period
    add(0, 4, 1, 1, TT_TAPS_JAKES, 0, TT_TAP_F32, 0, 0);
    add(0, 33, 1, 2, TT_TAPS_HOLD, 12, TT_TAP_F32, 0, 2);      // hears two gNB streams
    add(1, 24, 2, 2, TT_TAPS_JAKES, 0, TT_TAP_F32, 0, 0);
    add(1, 64, 2, 1, TT_TAPS_LINEAR, 256, TT_TAP_F32, 0, 0);
    add(1, 1, 1, 2, TT_TAPS_HOLD, 1, TT_TAP_F32, 0, 0);        // one tap, a snapshot per sample
    return v;
}

void set_all_taps(tt_channel* ch, Ue& u)
{
    const int64_t samples = kTotal[u.cfg.cell];
    std::mt19937 g(7 + u.id);
    std::normal_distribution<float> nd(0.f, 0.3f);
    if (u.cfg.mode == TT_TAPS_JAKES) {
        for (int d = 0; d < 2; ++d) {
            const int nrx = d == TT_DL ? u.cfg.n_rx : u.ul_rx, ntx = d == TT_DL ? u.dl_tx : u.cfg.n_tx;
            const int L = u.cfg.n_taps;
            std::vector<double> pdp(L, 1.0 / L), th((size_t)nrx * ntx * L), ph((size_t)nrx * ntx * L * 16);
            for (double& x : th)
                x = nd(g);
            for (double& x : ph)
                x = nd(g) * 3.0;
            OK(tt_channel_set_jakes(ch, u.id, d, d ? 480.0 : 35.0, pdp.data(), th.data(), ph.data()));
        }
        return;
    }
    // a snapshot per period up to the samples the run uses, in blocks the ring holds
    const int64_t last = samples / u.cfg.snapshot_period + 2;
    for (int d = 0; d < 2; ++d) {
        const int nrx = d == TT_DL ? u.cfg.n_rx : u.ul_rx, ntx = d == TT_DL ? u.dl_tx : u.cfg.n_tx;
        const int64_t per = (int64_t)nrx * ntx * u.cfg.n_taps;
        const int tb = u.cfg.tap_fmt == TT_TAP_F16 ? 4 : 8;
        const int64_t cap = u.cfg.ring_snapshots;
        for (int64_t k0 = std::max<int64_t>(0, last + 1 - cap); k0 <= last; k0 += 512) {
            const int32_t count = (int32_t)std::min<int64_t>(512, last + 1 - k0);
            std::vector<unsigned char> buf((size_t)count * per * tb);
            for (size_t i = 0; i < buf.size(); i += 4) {
                const float f = nd(g);
                std::memcpy(&buf[i], &f, 4);
                if (tb == 4) {  // f16 pairs: keep the values finite and small
                    buf[i + 1] = 0x30;
                    buf[i + 3] = 0x30;
                }
            }
            OK(tt_channel_set_taps(ch, u.id, d, k0, count, buf.data()));
        }
    }
}

tt_tuning tuning(int R, int ulg, int red, int dlg, int pf, int persist, int graph, int sub = 0)
{
    tt_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.outputs_per_lane = R;
    t.ul_group = ulg;
    t.ul_reduce = red;
    t.dl_group = dlg;
    t.prefetch = pf;
    t.persist = persist;
    t.graph = graph;
    t.dl_subtiles = sub;
    return t;
}

tt_channel* make_channel(int max_ues, int64_t budget)
{
    tt_cell_cfg cells[kCells];
    std::memset(cells, 0, sizeof(cells));
    for (int c = 0; c < kCells; ++c) {
        cells[c].sample_rate_hz = kRate[c];
        cells[c].n_ant = kAnt[c];
        cells[c].max_samples = kMax[c];
        cells[c].ul_sigma = 0.02f;
        for (int a = 0; a < TT_MAX_ANT; ++a)
            cells[c].ul_noise_off[a] = 1000 * c + a;
    }
    std::vector<uint16_t> pool(2 * 4096, 0x2c00);
    tt_channel_cfg cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.max_ues = max_ues;
    cfg.hbm_budget_bytes = budget;
    cfg.n_cells = kCells;
    cfg.cells = cells;
    cfg.iq_fmt = TT_IQ_CI16;
    cfg.noise_pool = pool.data();
    cfg.noise_pool_len = 4096;
    tt_channel* ch = nullptr;
    OK(tt_channel_create(&cfg, &ch));
    return ch;
}

// Slots through every apply form under one schedule.
void run_schedules(int64_t* clock_out)
{
    std::vector<Ue> ues = make_ues();
    tt_channel* ch = make_channel(16, 64 << 20);
    for (Ue& u : ues) {
        OK(tt_channel_add_ue(ch, &u.cfg, &u.id));
        set_all_taps(ch, u);
    }
    // per-UE input/output buffers at the largest call, gNB streams per cell
    std::vector<void*> dlx, dly, ulx;
    void* gnb[kCells];
    void* z[kCells];
    for (int c = 0; c < kCells; ++c) {
        gnb[c] = dev((size_t)kAnt[c] * kMax[c] * 4);
        z[c] = dev((size_t)kAnt[c] * kMax[c] * 4);
    }
    for (Ue& u : ues) {
        const int N = kMax[u.cfg.cell];
        dlx.push_back(u.cfg.dl_tx_streams > 0 ? dev((size_t)u.dl_tx * N * 4) : gnb[u.cfg.cell]);
        dly.push_back(dev((size_t)u.cfg.n_rx * N * 4));
        ulx.push_back(dev((size_t)u.cfg.n_tx * N * 4));
    }
    const tt_tuning sched[] = {
        tuning(0, 0, 0, 0, 0, 0, 0),        tuning(1, 1, 1, 1, 2, -1, 2, 4), tuning(2, 4, 2, 4, 1, -1, 2, 2),
        tuning(4, 2, 1, 2, 1, 2, 2, 2),     tuning(8, 8, 2, 8, 2, 1, 1, 2),  tuning(4, 16, 2, 1, 2, -1, 1, 4),
    };
    const int sizes[][kCells] = {{4096, 8192}, {1000, 333}, {4096, 1}, {17, 8191}, {256, 512}};
    int step = 0;
    for (const tt_tuning& t0 : sched) {
        tt_tuning t = t0;
        if (step % 2)  // per-class schedules on some rounds
            for (int m = 0; m < 3; ++m)
                for (int b = 0; b < 4; ++b)
                    for (int r = 0; r < TT_MAX_ANT; ++r)
                        t.outputs_by_class[m][b][r] = 1 << ((m + b + r) % 4);
        OK(tt_channel_set_tuning(ch, &t));
        for (const auto& sz : sizes) {
            std::vector<int32_t> ids, ns;
            std::vector<const void*> xs, uxs;
            std::vector<void*> ys;
            for (size_t i = 0; i < ues.size(); ++i) {
                ids.push_back(ues[i].id);
                ns.push_back(sz[ues[i].cfg.cell]);
                xs.push_back(dlx[i]);
                ys.push_back(dly[i]);
                uxs.push_back(ulx[i]);
            }
            const int32_t cell_samples[kCells] = {sz[0], sz[1]};
            switch (step % 4) {
            case 0: {  // fused slot
                tt_slot s;
                std::memset(&s, 0, sizeof(s));
                s.n_dl = (int32_t)ids.size();
                s.dl_ue = ids.data();
                s.dl_x = xs.data();
                s.dl_y = ys.data();
                s.n_ul = (int32_t)ids.size();
                s.ul_ue = ids.data();
                s.ul_x = uxs.data();
                s.ul_z = z;
                s.cell_samples = cell_samples;
                OK(tt_channel_apply_slot(ch, &s));
                break;
            }
            case 1: {  // prepared, then launched
                tt_slot s;
                std::memset(&s, 0, sizeof(s));
                s.n_dl = (int32_t)ids.size();
                s.dl_ue = ids.data();
                s.dl_x = xs.data();
                s.dl_y = ys.data();
                s.n_ul = (int32_t)ids.size();
                s.ul_ue = ids.data();
                s.ul_x = uxs.data();
                s.ul_z = z;
                s.cell_samples = cell_samples;
                OK(tt_channel_prepare_slot(ch, &s));
                REFUSED(tt_channel_set_tuning(ch, &t), TT_E_STATE);
                OK(tt_channel_launch_prepared(ch));
                REFUSED(tt_channel_launch_prepared(ch), TT_E_STATE);
                break;
            }
            default: {  // separate DL and per-cell UL calls (allocation-free UL on odd steps)
                // DL per cell: the calls of one cell share N
                for (int c = 0; c < kCells; ++c) {
                    std::vector<int32_t> ci, cn;
                    std::vector<const void*> cx;
                    std::vector<void*> cy;
                    std::vector<const void*> cu;
                    for (size_t i = 0; i < ues.size(); ++i)
                        if (ues[i].cfg.cell == c) {
                            ci.push_back(ids[i]);
                            cn.push_back(ns[i]);
                            cx.push_back(xs[i]);
                            cy.push_back(ys[i]);
                            cu.push_back(uxs[i]);
                        }
                    OK(tt_channel_apply_dl(ch, (int32_t)ci.size(), ci.data(), cn.data(), cx.data(), cy.data()));
                    const uint32_t both = TT_UL_BEGIN | TT_UL_END;
                    if (step % 4 == 3)
                        OK(tt_channel_apply_ul_noalloc(ch, c, sz[c], (int32_t)ci.size(), ci.data(), cu.data(), z[c],
                                                       both));
                    else
                        OK(tt_channel_apply_ul(ch, c, sz[c], (int32_t)ci.size(), ci.data(), cu.data(), z[c], both));
                }
            }
            }
            ++step;
        }
        OK(tt_channel_sync(ch));
    }
    // refusals: longer-than-max calls for sparse and Jakes downlinks, bad ids, bad rings
    {
        const int32_t sparse_ue = ues[2].id, jakes_ue = ues[3].id;
        const int32_t n_long = kMax[0] + 1;
        void* big_x = dev((size_t)n_long * 4);
        void* big_y = dev((size_t)n_long * 4);
        const void* bx[] = {big_x};
        void* by[] = {big_y};
        REFUSED(tt_channel_apply_dl(ch, 1, &sparse_ue, &n_long, bx, by), TT_E_INVALID);
        REFUSED(tt_channel_apply_dl(ch, 1, &jakes_ue, &n_long, bx, by), TT_E_INVALID);
        REFUSED(tt_channel_apply_ul(ch, 0, n_long, 1, &jakes_ue, bx, z[0], TT_UL_BEGIN | TT_UL_END), TT_E_INVALID);
        const int32_t bad = 99, one = 10;
        REFUSED(tt_channel_apply_dl(ch, 1, &bad, &one, bx, by), TT_E_INVALID);
        std::vector<float> t((size_t)4096 * 8 * 2);
        REFUSED(tt_channel_set_taps(ch, ues[0].id, TT_DL, 0, 4096, t.data()), TT_E_INVALID);
        tt_tuning bad_sub = tuning(4, 8, 2, 1, 2, -1, 2, 3);  // lane tiles must be 1, 2 or 4
        REFUSED(tt_channel_set_tuning(ch, &bad_sub), TT_E_INVALID);
        hipFree(big_x);
        hipFree(big_y);
    }
    // Jakes anchor tables: a faster Doppler (closer anchors) grows the table
    {
        Ue& u = ues[3];
        std::vector<double> pdp(u.cfg.n_taps, 0.25), th(u.cfg.n_taps, 0.1), ph((size_t)u.cfg.n_taps * 16, 0.3);
        OK(tt_channel_set_jakes(ch, u.id, TT_DL, 2500.0, pdp.data(), th.data(), ph.data()));
        const int32_t n = 3000;
        const void* x[] = {dlx[3]};
        void* y[] = {dly[3]};
        OK(tt_channel_apply_dl(ch, 1, &u.id, &n, x, y));
        OK(tt_channel_set_jakes(ch, u.id, TT_DL, 1.0, pdp.data(), th.data(), ph.data()));
        OK(tt_channel_apply_dl(ch, 1, &u.id, &n, x, y));
    }
    // kernel timing and counters
    {
        OK(tt_channel_enable_kernel_timing(ch, 1));
        const int32_t n = 2048;
        std::vector<int32_t> ids;
        std::vector<const void*> xs;
        std::vector<void*> ys;
        for (size_t i = 0; i < ues.size(); ++i)
            if (ues[i].cfg.cell == 0) {
                ids.push_back(ues[i].id);
                xs.push_back(dlx[i]);
                ys.push_back(dly[i]);
            }
        std::vector<int32_t> ns(ids.size(), n);
        OK(tt_channel_apply_dl(ch, (int32_t)ids.size(), ids.data(), ns.data(), xs.data(), ys.data()));
        double ms = 0;
        int64_t launches = 0;
        for (int k = 0; k < 3; ++k)
            OK(tt_channel_kernel_time_kind(ch, k, &ms, &launches));
        REFUSED(tt_channel_kernel_time_kind(ch, 3, &ms, &launches), TT_E_INVALID);
        tt_stats st;
        OK(tt_channel_get_stats(ch, &st));
        expect(st.active_ues == (int32_t)ues.size(), "active UEs", __LINE__);
    }
    // remove and re-add (deferred releases, anchor tables returned)
    for (int r = 0; r < 3; ++r)
        for (Ue& u : ues) {
            OK(tt_channel_remove_ue(ch, u.id));
            OK(tt_channel_add_ue(ch, &u.cfg, &u.id));
            set_all_taps(ch, u);
        }
    *clock_out = step;
    OK(tt_channel_destroy(ch));
    for (void* p : dly)
        hipFree(p);
    for (size_t i = 0; i < ues.size(); ++i)
        if (ues[i].cfg.dl_tx_streams > 0)
            hipFree(dlx[i]);
    for (void* p : ulx)
        hipFree(p);
    for (int c = 0; c < kCells; ++c) {
        hipFree(gnb[c]);
        hipFree(z[c]);
    }
}

// Admission by footprint: a small arena admits part of the UEs; Jakes tables
// that do not fit are refused without changing the link.
void run_admission()
{
    std::vector<Ue> ues = make_ues();
    tt_channel* ch = make_channel(4, 16 << 20);
    int admitted = 0;
    for (Ue& u : ues) {
        const tt_status s = tt_channel_add_ue(ch, &u.cfg, &u.id);
        expect(s == TT_OK || s == TT_E_ADMIT, "admission status", __LINE__);
        admitted += s == TT_OK;
        if (s != TT_OK)
            u.id = -1;
    }
    expect(admitted >= 1 && admitted <= 4, "some admitted", __LINE__);
    for (Ue& u : ues)
        if (u.id >= 0)
            OK(tt_channel_remove_ue(ch, u.id));
    OK(tt_channel_destroy(ch));
}

// The serving loop with joins, leaves, queueing, plain and copied taps.
void run_server(int plain, int copy_taps)
{
    std::vector<Ue> ues = make_ues();
    tt_channel* ch = make_channel(8, 64 << 20);
    const int n_slots = 24, x_slots = 3, y_slots = 2, z_slots = 2;
    const int32_t N[kCells] = {2048, 4096};
    std::vector<tt_stream> st(ues.size());
    std::vector<void*> bufs;
    std::vector<std::vector<double>> host;  // Jakes parameters
    host.reserve(ues.size() * 6);
    for (size_t i = 0; i < ues.size(); ++i) {
        Ue& u = ues[i];
        tt_stream& s = st[i];
        std::memset(&s, 0, sizeof(s));
        s.cfg = u.cfg;
        s.arrive_slot = (int64_t)(i % 4) * 3;
        s.session_slots = i % 3 == 0 ? 5 : 0;
        const int n = N[u.cfg.cell];
        s.ul_x = dev((size_t)x_slots * u.cfg.n_tx * n * 4);
        bufs.push_back(const_cast<void*>(s.ul_x));
        s.x_slots = x_slots;
        s.dl_y = dev((size_t)y_slots * u.cfg.n_rx * n * 4);
        bufs.push_back(s.dl_y);
        s.y_slots = y_slots;
        if (u.cfg.mode == TT_TAPS_JAKES) {
            for (int d = 0; d < 2; ++d) {
                const int nrx = d == TT_DL ? u.cfg.n_rx : u.ul_rx, ntx = d == TT_DL ? u.dl_tx : u.cfg.n_tx;
                host.emplace_back(u.cfg.n_taps, 1.0 / u.cfg.n_taps);
                s.pdp[d] = host.back().data();
                host.emplace_back((size_t)nrx * ntx * u.cfg.n_taps, 0.2);
                s.theta[d] = host.back().data();
                host.emplace_back((size_t)nrx * ntx * u.cfg.n_taps * 16, 0.7);
                s.phi[d] = host.back().data();
                s.doppler_hz[d] = 100.0 * (d + 1);
            }
        } else {
            s.tap_len = 40;
            for (int d = 0; d < 2; ++d) {
                const int nrx = d == TT_DL ? u.cfg.n_rx : u.ul_rx, ntx = d == TT_DL ? u.dl_tx : u.cfg.n_tx;
                const size_t bytes = (size_t)(s.tap_len + 1) * nrx * ntx * u.cfg.n_taps *
                                     (u.cfg.tap_fmt == TT_TAP_F16 ? 4 : 8);
                s.taps[d] = dev(bytes);
                bufs.push_back(const_cast<void*>(s.taps[d]));
            }
        }
    }
    void* dl_x[kCells];
    void* ul_z[kCells];
    for (int c = 0; c < kCells; ++c) {
        dl_x[c] = dev((size_t)x_slots * kAnt[c] * N[c] * 4);
        ul_z[c] = dev((size_t)z_slots * kAnt[c] * N[c] * 4);
    }
    std::vector<double> lat(n_slots);
    std::vector<int32_t> active(n_slots);
    std::vector<int64_t> adm(ues.size()), lv(ues.size());
    tt_serve_cfg cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.n_slots = n_slots;
    cfg.max_active = 5;
    const void* dx[kCells] = {dl_x[0], dl_x[1]};
    cfg.dl_x = dx;
    cfg.x_slots = x_slots;
    cfg.ul_z = ul_z;
    cfg.z_slots = z_slots;
    cfg.cell_samples = N;
    cfg.plain = plain;
    cfg.copy_taps = copy_taps;
    cfg.lat_us = lat.data();
    cfg.active = active.data();
    cfg.admit_slot = adm.data();
    cfg.leave_slot = lv.data();
    tt_server* srv = nullptr;
    // the multi-gNB UE's DL input is not the cell's stream: the loop refuses it
    tt_server* bad = nullptr;
    REFUSED(tt_server_create(ch, &cfg, (int32_t)st.size(), st.data(), &bad), TT_E_INVALID);
    st.erase(st.begin() + 4);
    OK(tt_server_create(ch, &cfg, (int32_t)st.size(), st.data(), &srv));
    OK(tt_server_run(srv, 10));
    OK(tt_server_run(srv, n_slots - 10));
    REFUSED(tt_server_run(srv, 1), TT_E_INVALID);
    tt_serve_stats ss;
    OK(tt_server_stats(srv, &ss, 1));
    expect(ss.slots == n_slots && ss.admitted >= 4, "served slots", __LINE__);
    OK(tt_server_destroy(srv));
    OK(tt_channel_destroy(ch));
    for (void* p : bufs)
        hipFree(p);
    for (int c = 0; c < kCells; ++c) {
        hipFree(dl_x[c]);
        hipFree(ul_z[c]);
    }
}

// The host IQ pipeline over the UEs of cell 0 that hear only their cell.
void run_io()
{
    std::vector<Ue> ues = make_ues();
    tt_channel* ch = make_channel(8, 64 << 20);
    std::vector<int32_t> ids;
    for (Ue& u : ues)
        if (u.cfg.cell == 0 && u.cfg.dl_tx_streams == 0) {
            OK(tt_channel_add_ue(ch, &u.cfg, &u.id));
            set_all_taps(ch, u);
            ids.push_back(u.id);
        }
    tt_io_cfg cfg;
    std::memset(&cfg, 0, sizeof(cfg));
    cfg.cell = 0;
    cfg.n_ues = (int32_t)ids.size();
    cfg.ue = ids.data();
    cfg.n_samples = 2048;
    cfg.depth = 3;
    tt_io* io = nullptr;
    OK(tt_io_create(ch, &cfg, &io));
    for (int s = 0; s < 9; ++s) {
        const int b = s % 3;
        if (s >= 3) {
            double us = 0;
            OK(tt_io_wait(io, b, &us));
        }
        void *in = nullptr, *out = nullptr;
        int64_t ib = 0, ob = 0;
        OK(tt_io_buffers(io, b, &in, &ib, &out, &ob));
        std::memset(in, 0, (size_t)ib);
        OK(tt_io_submit(io, b));
        int32_t inflight = 0;
        OK(tt_io_poll(io, &inflight));
    }
    OK(tt_io_destroy(io));
    OK(tt_channel_destroy(ch));
}

}  // namespace

int main()
{
    int64_t steps = 0;
    run_schedules(&steps);
    run_admission();
    for (int plain = 0; plain < 2; ++plain)
        for (int copy = 0; copy < 2; ++copy)
            run_server(plain, copy);
    run_io();
    const int64_t live = hip_model_live_blocks();
    expect(live == 0, "every device and pinned allocation returned", __LINE__);
    std::printf("host model: %lld slot steps, %lld kernel launches checked, %lld allocations live, %d failures\n",
                (long long)steps, (long long)hip_model_launches(), (long long)live, g_fail);
    return g_fail == 0 && live == 0 ? 0 : 1;
}
