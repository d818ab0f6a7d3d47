// Slot-paced serving loop over a channel: admission by arena footprint,
// joins queued in arrival order, device-resident tap and IQ sources, one
// batched DL+UL call per slot, and per-slot submit-to-completion latency.
#include "tt_internal.h"
#include "tt_channel.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <numeric>
#include <string>
#include <vector>

namespace {

using Clock = std::chrono::steady_clock;

// A paced slot whose launch starts more than this fraction of the slot period
// after its tick counts as a late start.
constexpr double kLateFraction = 0.1;

double us_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::micro>(b - a).count();
}

struct StreamState {
    int32_t ue = -1;
    int64_t admit = -1, leave = -1;
    int64_t served = 0;  // slots served so far
};

struct Inflight {
    int64_t slot;
    hipEvent_t ev;
    Clock::time_point t_ref;  // the slot's tick when paced, else its submission
};

double percentile(std::vector<double> v, double p)
{
    if (v.empty())
        return 0.0;
    std::sort(v.begin(), v.end());
    size_t k = (size_t)std::ceil(p / 100.0 * (double)v.size());  // nearest rank
    if (k < 1)
        k = 1;
    return v[std::min(k, v.size()) - 1];
}

tt_status bad(const char* m)
{
    tt::set_error(m);
    return TT_E_INVALID;
}


}  // namespace

struct tt_server {
    tt_channel* ch = nullptr;
    tt_serve_cfg cfg{};
    std::vector<tt_stream> streams;
    std::vector<int32_t> cell_n;
    std::vector<const void*> dl_x_cells;
    std::vector<void*> ul_z_cells;
    const tt_cell_cfg* cells = nullptr;
    int n_cells = 0;
    int64_t sb = 4;
    std::vector<int> order;
    size_t next_arrival = 0;
    std::deque<int> queue;
    std::vector<StreamState> ss;
    std::vector<int> active;
    std::vector<double> lat;
    std::vector<int32_t> act;
    int64_t slot = 0;          // next slot index
    int64_t stat_from = 0;     // first slot of the current statistics window
    tt_serve_stats acc{};      // counters of the window
    Clock::time_point t_first{}, t_last{};
    bool have_first = false;
    double host_us_sum = 0.0;
    double build_us_sum = 0.0, wait_us_sum = 0.0;  // building slots ahead; blocked on the GPU
    double lag_max_us = 0.0;   // largest delay of a paced slot's launch after its tick
    int64_t last_calls = 1;    // descriptor-consuming channel calls of the previous slot
    bool staged_ok = false;    // the next slot is prepared in the channel, awaiting its launch
    int64_t staged_uses = 0;   // descriptor uses of building it
    std::deque<Inflight> inflight;
    tt_status rc = TT_OK;
    // scratch reused every slot
    std::vector<std::vector<tt_taps_src>> pieces;  // ingest entries, one list per run of the pools
    std::vector<int32_t> dl_ue, ul_ue;
    std::vector<const void*> dl_x, ul_x, dl_taps, ul_taps;
    std::vector<const void*> ext[2];  // per active position: zero-copy snapshots or nullptr
    std::vector<void*> dl_y, ul_z;

    void poll(bool block)
    {
        while (!inflight.empty()) {
            Inflight& f = inflight.front();
            hipError_t q = block ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
            if (q == hipErrorNotReady)
                return;
            const Clock::time_point now = Clock::now();
            if (q != hipSuccess && rc == TT_OK) {
                rc = TT_E_DEVICE;
                tt::set_error("tt_server: device error while waiting for a slot");
            }
            lat[f.slot] = us_between(f.t_ref, now);
            t_last = now;
            inflight.pop_front();
        }
    }

    void poll_one_blocking()
    {
        Inflight& f = inflight.front();
        hipError_t q = hipEventSynchronize(f.ev);
        const Clock::time_point now = Clock::now();
        if (q != hipSuccess && rc == TT_OK) {
            rc = TT_E_DEVICE;
            tt::set_error("tt_server: device error while waiting for a slot");
        }
        lat[f.slot] = us_between(f.t_ref, now);
        t_last = now;
        inflight.pop_front();
    }

    tt_status retire_finished(int64_t s)
    {
        for (size_t a = 0; a < active.size();) {
            const int i = active[a];
            const tt_stream& sp = streams[i];
            if (sp.session_slots > 0 && s >= ss[i].admit + sp.session_slots) {
                tt_status r = tt_channel_remove_ue(ch, ss[i].ue);
                if (r != TT_OK)
                    return r;
                ss[i].leave = s;
                ++acc.left;
                active.erase(active.begin() + a);
            } else {
                ++a;
            }
        }
        return TT_OK;
    }

    tt_status admit(int64_t s)
    {
        while (next_arrival < order.size() && streams[order[next_arrival]].arrive_slot <= s)
            queue.push_back(order[next_arrival++]);
        while (!queue.empty() && (int)active.size() < cfg.max_active) {
            const int i = queue.front();
            const tt_stream& sp = streams[i];
            int32_t id = -1;
            tt_status r = tt_channel_add_ue(ch, &sp.cfg, &id);
            if (r == TT_E_ADMIT)
                break;  // head of the queue waits for memory to free up
            if (r != TT_OK)
                return r;
            if (sp.cfg.mode == TT_TAPS_JAKES) {
                for (int d = 0; d < 2 && r == TT_OK; ++d)
                    r = tt_channel_set_jakes(ch, id, d, sp.doppler_hz[d], sp.pdp[d], sp.theta[d], sp.phi[d]);
                if (r == TT_E_ADMIT) {
                    // its anchor tables do not fit yet: it waits at the head of the queue
                    r = tt_channel_remove_ue(ch, id);
                    if (r != TT_OK)
                        return r;
                    break;
                }
                if (r != TT_OK)
                    return r;
            }
            ss[i] = StreamState();
            ss[i].ue = id;
            ss[i].admit = s;
            active.push_back(i);
            queue.pop_front();
            ++acc.admitted;
        }
        acc.max_queue = std::max<int64_t>(acc.max_queue, (int64_t)queue.size());
        return TT_OK;
    }

    // Snapshots for this slot: a zero-copy pointer into the pool when the
    // slot's range is contiguous there, else a copy into the UE's tap ring.
    tt_status ingest()
    {
        for (auto& v : pieces)
            v.clear();
        for (int d = 0; d < 2; ++d)
            ext[d].assign(active.size(), nullptr);
        for (size_t a = 0; a < active.size(); ++a) {
            const int i = active[a];
            const tt_stream& sp = streams[i];
            if (sp.cfg.mode == TT_TAPS_JAKES)
                continue;
            const int64_t N = cfg.cell_samples[sp.cfg.cell];
            if (N == 0)
                continue;
            const int64_t clock = ss[i].served * N;
            const int64_t P = sp.cfg.snapshot_period;
            const int64_t k_first = clock / P;
            const int64_t k_last = (clock + N - 1) / P + (sp.cfg.mode == TT_TAPS_LINEAR ? 1 : 0);
            const int64_t count = k_last - k_first + 1;
            for (int d = 0; d < 2; ++d) {
                const int n_tx = d == TT_DL ? cells[sp.cfg.cell].n_ant : sp.cfg.n_tx;
                const int n_rx = d == TT_DL ? sp.cfg.n_rx : cells[sp.cfg.cell].n_ant;
                const int64_t per_bytes =
                    (int64_t)n_rx * n_tx * sp.cfg.n_taps * (sp.cfg.tap_fmt == TT_TAP_F16 ? 4 : 8);
                const char* base = static_cast<const char*>(sp.taps[d]);
                const int64_t e0 = k_first % sp.tap_len;
                // entry tap_len repeats entry 0, so a run may end at index tap_len
                const int64_t first_run = std::min(count, sp.tap_len + 1 - e0);
                if (!cfg.copy_taps && !cfg.plain && first_run == count) {
                    ext[d][a] = base + e0 * per_bytes;
                    continue;
                }
                // contiguous runs through the pool, the p-th run of every
                // link in list p (a call lists each link once); a slot that
                // needs more snapshots than the pool holds wraps several times
                int64_t k = k_first, left = count;
                for (size_t p = 0; left > 0; ++p) {
                    const int64_t e = k % sp.tap_len;
                    const int64_t run = std::min(left, sp.tap_len + 1 - e);
                    if (pieces.size() <= p)
                        pieces.emplace_back();
                    pieces[p].push_back(tt_taps_src{ss[i].ue, d, k, (int32_t)run, base + e * per_bytes});
                    k += run;
                    left -= run;
                }
            }
        }
        tt_status r = TT_OK;
        for (size_t p = 0; p < pieces.size() && r == TT_OK; ++p)
            if (!pieces[p].empty())
                r = tt_channel_set_taps_device(ch, (int32_t)pieces[p].size(), pieces[p].data());
        return r;
    }

    tt_status apply(int64_t s, bool staged)
    {
        dl_ue.clear();
        ul_ue.clear();
        dl_x.clear();
        dl_y.clear();
        ul_x.clear();
        dl_taps.clear();
        ul_taps.clear();
        std::fill(ul_z.begin(), ul_z.end(), nullptr);
        for (size_t a = 0; a < active.size(); ++a) {
            const int i = active[a];
            const tt_stream& sp = streams[i];
            dl_taps.push_back(ext[TT_DL][a]);
            ul_taps.push_back(ext[TT_UL][a]);
            const int c = sp.cfg.cell;
            const int64_t N = cfg.cell_samples[c];
            const int n_ant = cells[c].n_ant;
            dl_ue.push_back(ss[i].ue);
            dl_x.push_back(static_cast<const char*>(dl_x_cells[c]) + (s % cfg.x_slots) * n_ant * N * sb);
            dl_y.push_back(static_cast<char*>(sp.dl_y) + (s % sp.y_slots) * sp.cfg.n_rx * N * sb);
            ul_ue.push_back(ss[i].ue);
            ul_x.push_back(static_cast<const char*>(sp.ul_x) + (ss[i].served % sp.x_slots) * sp.cfg.n_tx * N * sb);
            ul_z[c] = static_cast<char*>(ul_z_cells[c]) + (s % cfg.z_slots) * n_ant * N * sb;
            acc.link_samples += N * (sp.cfg.n_rx + n_ant);
        }
        if (active.empty())
            return TT_OK;
        if (!cfg.plain) {
            tt_slot sl{};
            sl.n_dl = (int32_t)dl_ue.size();
            sl.dl_ue = dl_ue.data();
            sl.dl_x = dl_x.data();
            sl.dl_y = dl_y.data();
            sl.n_ul = (int32_t)ul_ue.size();
            sl.ul_ue = ul_ue.data();
            sl.ul_x = ul_x.data();
            sl.ul_z = ul_z.data();
            sl.cell_samples = cell_n.data();
            sl.dl_taps = dl_taps.data();
            sl.ul_taps = ul_taps.data();
            if (!staged)
                return tt_channel_apply_slot(ch, &sl);
            tt_status r = tt_channel_prepare_slot(ch, &sl);
            staged_ok = r == TT_OK;
            return r;
        }
        tt_status r = TT_OK;
        for (size_t a = 0; a < active.size() && r == TT_OK; ++a) {
            const int32_t N = cfg.cell_samples[streams[active[a]].cfg.cell];
            r = tt_channel_apply_dl(ch, 1, &dl_ue[a], &N, &dl_x[a], &dl_y[a]);
        }
        for (int c = 0; c < n_cells && r == TT_OK; ++c) {
            std::vector<size_t> mem;
            for (size_t a = 0; a < active.size(); ++a)
                if (streams[active[a]].cfg.cell == c)
                    mem.push_back(a);
            std::sort(mem.begin(), mem.end(), [&](size_t x, size_t y) { return ul_ue[x] < ul_ue[y]; });
            for (size_t k = 0; k < mem.size() && r == TT_OK; ++k) {
                const uint32_t fl = (k == 0 ? (uint32_t)TT_UL_BEGIN : 0u) | (k + 1 == mem.size() ? (uint32_t)TT_UL_END : 0u);
                r = tt_channel_apply_ul(ch, c, cfg.cell_samples[c], 1, &ul_ue[mem[k]], &ul_x[mem[k]], ul_z[c], fl);
            }
        }
        return r;
    }

    // Control-plane work of slot s: retire, admit, snapshot ingest and the
    // slot's batch.  With staged = true the batch is only prepared in the
    // channel (descriptors built, clocks advanced); its kernels are enqueued
    // at the slot's tick by tt_channel_launch_prepared.
    tt_status build(int64_t s, bool staged)
    {
        tt_status r = retire_finished(s);
        if (r == TT_OK)
            r = admit(s);
        if (r == TT_OK)
            r = ingest();
        if (r == TT_OK)
            r = apply(s, staged);
        if (r != TT_OK)
            return r;
        for (int i : active)
            ++ss[i].served;
        act[s] = (int32_t)active.size();
        acc.ue_slots += (int64_t)active.size();
        return TT_OK;
    }

    tt_status run(int32_t n)
    {
        if (rc != TT_OK)
            return rc;
        if (n < 0 || slot + n > cfg.n_slots)
            return bad("tt_server_run: past the configured n_slots");
        // Batched slots are built one slot ahead: slot s + 1's control plane
        // runs while slot s is on the GPU, so a slot's latency, timed from its
        // tick, holds only its launch and its GPU work.  Plain per-UE calls are
        // built at the tick.
        const bool ahead = !cfg.plain;
        auto stage = [&](int64_t s) {
            const Clock::time_point b0 = Clock::now();
            const int64_t u0 = tt::channel_desc_uses(ch);
            staged_ok = false;
            tt_status r = build(s, true);
            staged_uses = tt::channel_desc_uses(ch) - u0;
            build_us_sum += us_between(b0, Clock::now());
            return r;
        };
        if (ahead && n > 0) {
            rc = stage(slot);
            if (rc != TT_OK)
                return rc;
        }
        const Clock::time_point t0 = Clock::now();
        for (int32_t j = 0; j < n && rc == TT_OK; ++j, ++slot) {
            const int64_t s = slot;
            const bool paced = cfg.slot_us > 0.0;
            Clock::time_point tick{};
            if (paced) {
                tick = t0 + std::chrono::duration_cast<Clock::duration>(
                                std::chrono::duration<double, std::micro>((double)j * cfg.slot_us));
                while (Clock::now() < tick)
                    poll(false);
            }
            // A slot's completion is the channel's own end-of-call event (one
            // marker per slot).  The channel re-records an event after
            // channel_event_depth() further descriptor uses, so earlier slots
            // are observed before this one can reuse their events (a slot
            // built ahead counts as one more in flight).
            const Clock::time_point w0 = Clock::now();
            while (!inflight.empty() &&
                   (int64_t)(inflight.size() + (ahead ? 2 : 1)) * last_calls > tt::channel_event_depth())
                poll_one_blocking();
            const Clock::time_point t_sub = Clock::now();
            wait_us_sum += us_between(w0, t_sub);
            // A paced slot's latency runs from its tick: a launch held back
            // past the tick (the previous slot's build, a full event window)
            // counts against the budget.
            const Clock::time_point t_ref = paced ? tick : t_sub;
            if (paced) {
                const double lag = us_between(tick, t_sub);
                lag_max_us = std::max(lag_max_us, lag);
                if (lag > kLateFraction * cfg.slot_us)
                    ++acc.late_starts;
            }
            if (!have_first) {
                t_first = t_sub;
                have_first = true;
            }
            int64_t uses = 0;
            tt_status r = TT_OK;
            if (ahead) {
                if (staged_ok)
                    r = tt_channel_launch_prepared(ch);
                staged_ok = false;
                uses = staged_uses;
            } else {
                const int64_t uses0 = tt::channel_desc_uses(ch);
                r = build(s, false);
                uses = tt::channel_desc_uses(ch) - uses0;
            }
            if (r != TT_OK) {
                rc = r;
                break;
            }
            last_calls = std::max<int64_t>(1, uses);
            if (uses > 0) {
                inflight.push_back(Inflight{s, tt::channel_last_event(ch), t_ref});
            } else {  // no GPU work this slot
                lat[s] = us_between(t_ref, Clock::now());
            }
            host_us_sum += us_between(t_sub, Clock::now());
            ++acc.slots;
            if (ahead && j + 1 < n) {
                r = stage(s + 1);
                if (r != TT_OK) {
                    rc = r;
                    ++slot;
                    break;
                }
            }
            poll(false);
        }
        poll(true);
        return rc;
    }

    void stats(tt_serve_stats* st, bool reset)
    {
        tt_serve_stats out = acc;
        std::vector<double> all, full;
        double sum = 0.0;
        const double budget = cfg.slot_us > 0.0 ? cfg.slot_us : 500.0;
        out.max_active = 0;
        out.min_active = 0;
        bool first = true;
        for (int64_t s = stat_from; s < slot; ++s) {
            out.max_active = std::max(out.max_active, act[s]);
            out.min_active = first ? act[s] : std::min(out.min_active, act[s]);
            first = false;
            if (lat[s] < 0.0)
                continue;
            all.push_back(lat[s]);
            sum += lat[s];
            if (lat[s] > budget)
                ++out.misses;
            if (act[s] == cfg.max_active) {
                full.push_back(lat[s]);
                ++out.full_slots;
            }
        }
        out.lat_p50_us = percentile(all, 50.0);
        out.lat_p99_us = percentile(all, 99.0);
        out.lat_max_us = all.empty() ? 0.0 : *std::max_element(all.begin(), all.end());
        out.lat_mean_us = all.empty() ? 0.0 : sum / (double)all.size();
        out.lat_p99_full_us = percentile(full, 99.0);
        out.wall_s = have_first ? std::chrono::duration<double>(t_last - t_first).count() : 0.0;
        out.queued_end = (int64_t)queue.size() + (int64_t)(order.size() - next_arrival);
        out.host_us_mean = acc.slots ? host_us_sum / (double)acc.slots : 0.0;
        out.build_us_mean = acc.slots ? build_us_sum / (double)acc.slots : 0.0;
        out.window_wait_us_mean = acc.slots ? wait_us_sum / (double)acc.slots : 0.0;
        out.start_lag_max_us = lag_max_us;
        *st = out;
        if (cfg.lat_us)
            std::memcpy(cfg.lat_us, lat.data(), sizeof(double) * lat.size());
        if (cfg.active)
            std::memcpy(cfg.active, act.data(), sizeof(int32_t) * act.size());
        if (cfg.admit_slot)
            for (size_t i = 0; i < ss.size(); ++i)
                cfg.admit_slot[i] = ss[i].admit;
        if (cfg.leave_slot)
            for (size_t i = 0; i < ss.size(); ++i)
                cfg.leave_slot[i] = ss[i].leave;
        if (reset) {
            acc = tt_serve_stats{};
            host_us_sum = 0.0;
            build_us_sum = wait_us_sum = 0.0;
            lag_max_us = 0.0;
            stat_from = slot;
            have_first = false;
        }
    }
};

extern "C" {

tt_status tt_server_create(tt_channel* ch, const tt_serve_cfg* cfg, int32_t n, const tt_stream* streams,
                           tt_server** out)
{
    if (!ch || !cfg || !out || n < 0 || (n > 0 && !streams))
        return bad("tt_server_create: null argument");
    *out = nullptr;
    int n_cells = 0;
    const tt_cell_cfg* cells = tt::channel_cells(ch, &n_cells);
    if (cfg->n_slots < 0 || cfg->max_active < 1 || !cfg->cell_samples || cfg->x_slots < 1 || cfg->z_slots < 1 ||
        !cfg->dl_x || !cfg->ul_z)
        return bad("tt_server_create: bad loop configuration");
    for (int c = 0; c < n_cells; ++c)
        if (cfg->cell_samples[c] < 0 || cfg->cell_samples[c] > cells[c].max_samples)
            return bad("tt_server_create: cell_samples out of range");
    for (int i = 0; i < n; ++i) {
        const tt_stream& s = streams[i];
        if (s.cfg.cell < 0 || s.cfg.cell >= n_cells)
            return bad("tt_server_create: stream cell out of range");
        if (!s.ul_x || s.x_slots < 1 || !s.dl_y || s.y_slots < 1)
            return bad("tt_server_create: stream IQ buffers missing");
        if (!cfg->dl_x[s.cfg.cell] || !cfg->ul_z[s.cfg.cell])
            return bad("tt_server_create: cell IQ buffers missing");
        // every served UE hears its cell's DL stream [n_ant][N]; stacked
        // streams of several gNBs would need an input of their own
        if (s.cfg.dl_tx_streams != 0)
            return bad("tt_server_create: streams with dl_tx_streams are not served by the loop");
        if (s.cfg.mode == TT_TAPS_JAKES) {
            for (int d = 0; d < 2; ++d)
                if (!s.pdp[d] || !s.theta[d] || !s.phi[d])
                    return bad("tt_server_create: Jakes parameters missing");
        } else if (!s.taps[0] || !s.taps[1] || s.tap_len < 1 || s.cfg.snapshot_period < 1) {
            return bad("tt_server_create: tap pools missing");
        }
    }
    tt_server* sv = new tt_server();
    sv->ch = ch;
    sv->cfg = *cfg;
    sv->cells = cells;
    sv->n_cells = n_cells;
    sv->sb = tt::channel_iq_fmt(ch) == TT_IQ_CI16 ? 4 : 8;
    sv->streams.assign(streams, streams + n);
    sv->cell_n.assign(cfg->cell_samples, cfg->cell_samples + n_cells);
    sv->dl_x_cells.assign(cfg->dl_x, cfg->dl_x + n_cells);
    sv->ul_z_cells.assign(cfg->ul_z, cfg->ul_z + n_cells);
    sv->cfg.cell_samples = sv->cell_n.data();
    sv->ul_z.assign(n_cells, nullptr);
    sv->order.resize(n);
    std::iota(sv->order.begin(), sv->order.end(), 0);
    std::stable_sort(sv->order.begin(), sv->order.end(),
                     [&](int a, int b) { return streams[a].arrive_slot < streams[b].arrive_slot; });
    sv->ss.resize(n);
    sv->lat.assign(cfg->n_slots, -1.0);
    sv->act.assign(cfg->n_slots, 0);
    *out = sv;
    return TT_OK;
}

tt_status tt_server_run(tt_server* srv, int32_t n_slots)
{
    if (!srv)
        return bad("tt_server_run: null server");
    return srv->run(n_slots);
}

tt_status tt_server_stats(tt_server* srv, tt_serve_stats* st, int32_t reset)
{
    if (!srv || !st)
        return bad("tt_server_stats: null argument");
    srv->stats(st, reset != 0);
    return TT_OK;
}

tt_status tt_server_destroy(tt_server* srv)
{
    if (!srv)
        return TT_OK;
    srv->poll(true);
    tt_status rc = TT_OK;
    for (int i : srv->active) {
        tt_status r = tt_channel_remove_ue(srv->ch, srv->ss[i].ue);
        srv->ss[i].leave = srv->slot;
        if (rc == TT_OK)
            rc = r;
    }
    if (srv->cfg.leave_slot)
        for (size_t i = 0; i < srv->ss.size(); ++i)
            srv->cfg.leave_slot[i] = srv->ss[i].leave;
    delete srv;
    return rc;
}

tt_status tt_serve(tt_channel* ch, const tt_serve_cfg* cfg, int32_t n, const tt_stream* streams, tt_serve_stats* st)
{
    if (!st)
        return bad("tt_serve: null stats");
    tt_server* sv = nullptr;
    tt_status rc = tt_server_create(ch, cfg, n, streams, &sv);
    if (rc != TT_OK)
        return rc;
    rc = sv->run(cfg->n_slots);
    sv->stats(st, false);
    tt_status r2 = tt_server_destroy(sv);
    return rc != TT_OK ? rc : r2;
}

}  // extern "C"
