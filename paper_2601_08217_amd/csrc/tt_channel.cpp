// Host runtime of the channel-emulation library: arena and admission, UE and
// link state (tap rings, Jakes parameters, histories, clocks), per-call
// descriptor tables, batching of UEs into launches, and the C ABI.
#include "tt_internal.h"
#include "tt_channel.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <string>
#include <vector>

using namespace tt;

namespace {

thread_local std::string g_err;

tt_status fail(tt_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

constexpr int64_t kAlign = 256;
constexpr int kMaxGroupsPerCell = 64;
constexpr int kDefaultGroup = 8;
constexpr int kDefaultDlGroup = 8;
constexpr int kDefaultR = 4;
constexpr int kDefaultPersist = 0;  // persistent grid off unless tuned
// Launch classes of a slot: one per (accumulator rows, outputs per lane R):
// class (n_rx - 1) * 4 + log2(R) + 1, so 1 .. 4 kMaxAnt.
constexpr int kClasses = 4 * kMaxAnt + 1;
int log2_r(int R) { return R >= 8 ? 3 : R >= 4 ? 2 : R >= 2 ? 1 : 0; }
int class_of(int n_rx, int R) { return (n_rx - 1) * 4 + log2_r(R) + 1; }
int class_nrx(int c) { return (c - 1) / 4 + 1; }
int class_r(int c) { return 1 << ((c - 1) % 4); }
// Shape classes of the per-class schedule: tap mode x tap-count bucket
// (L <= 8, <= 16, <= 32, <= 64) x receive antennas.
int taps_bucket(int L) { return L <= 8 ? 0 : L <= 16 ? 1 : L <= 32 ? 2 : 3; }
constexpr int kLdsLimit = 64 * 1024;
constexpr int kDescBufs = 16;
constexpr int kTimingPairs = 1024;   // event pairs created when kernel timing is enabled
constexpr size_t kDescMin = 256 * 1024;  // descriptor buffer floor (also the tap upload chunk)
constexpr double kJakesInterpBound = 1e-6;  // relative interpolation error between anchors

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

int64_t floor_div(int64_t a, int64_t b)
{
    if ((b & (b - 1)) == 0)  // b > 0 a power of two: an arithmetic shift floors
        return a >> __builtin_ctzll((unsigned long long)b);
    int64_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

int32_t mod_pool(int64_t a, int64_t npool)
{
    if ((npool & (npool - 1)) == 0)  // a power of two: the mask is the non-negative residue
        return (int32_t)(a & (npool - 1));
    int64_t r = a % npool;
    return (int32_t)(r < 0 ? r + npool : r);
}

// First-fit sub-allocator over one device allocation.
class Arena {
public:
    void init(int64_t cap)
    {
        cap_ = cap;
        used_ = 0;
        free_.clear();
        if (cap > 0)
            free_[0] = cap;
    }
    int64_t alloc(int64_t bytes)
    {
        bytes = align_up(bytes, kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > bytes)
                    free_[off + bytes] = sz - bytes;
                used_ += bytes;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        bytes = align_up(bytes, kAlign);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int64_t cap() const { return cap_; }
    int64_t used() const { return used_; }

private:
    int64_t cap_ = 0, used_ = 0;
    std::map<int64_t, int64_t> free_;
};

struct Link {
    int L = 0, n_tx = 0, n_rx = 0, mode = 0, tap_fmt = 0;
    int period = 1;          // P (HOLD/LINEAR) or anchor spacing K (JAKES)
    int nsel = 0;            // sparse top-n (0: every tap)
    int64_t clock = 0;
    int ring_cap = 0;
    int64_t ring_off = -1, jakes_off = -1, hist_off = -1;
    int64_t sel_off = -1;    // sparse: selected (H, D) pairs [sel_cap], then delays [sel_cap]
    int64_t sel_cap = 0;     // selection entries: one slot call of up to the cell's max_samples
    int64_t anc_off = -1;    // Jakes: anchor table [anc_cap][n_rx][n_tx][L] fp32 (allocated by set_jakes)
    int64_t anc_cap = 0, anc_bytes = 0;
    int64_t k_lo = 0, k_hi = 0;  // valid snapshots [k_lo, k_hi)
    bool jakes_set = false;
    // memos of the per-call schedule (the shape changes only with the period)
    mutable int lds_memo[12] = {};           // link_lds per (R = 1, 2, 4, 8; lane tiles 1, 2, 4) (0: not yet)
    mutable int64_t r_key = -1;               // (tuning generation, clock mod 8) of r_memo
    mutable int r_memo = 0;
    void forget_shape() const
    {
        for (int& m : lds_memo)
            m = 0;
        r_key = -1;
    }
    int per() const { return n_rx * n_tx * L; }
    int tap_bytes() const { return tap_fmt == TAP_F16 ? 4 : 8; }
};

struct Ue {
    bool active = false;
    tt_ue_cfg cfg{};
    int64_t off = -1, bytes = 0;
    Link link[2];
    int64_t m0 = 0;
};

struct DescBuf {
    char* host = nullptr;
    char* host_dev = nullptr;  // device view of the pinned host buffer
    char* dev = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    hipEvent_t uploaded = nullptr;  // upload of a staged slot, on the upload stream
    bool pending = false;
};

// A slot whose descriptors are built and staged in pinned memory, not yet
// enqueued: what the launch needs.
struct PreparedSlot {
    bool valid = false;
    DescBuf* db = nullptr;
    size_t off = 0;                     // staged descriptor bytes
    LaunchShape shape[kClasses];
    int njobs[kClasses] = {};
    size_t link_off[kClasses] = {}, job_off[kClasses] = {};
    size_t red_off = 0, red_sep_off = 0;
    int n_reds_sep = 0, red_max_n = 0, red_max_ant = 0;
    size_t sel_off = 0;                 // sparse selection pass: its entries
    int n_sel = 0, sel_blocks = 0;
    size_t anc_off = 0;                 // Jakes anchor pass: its entries
    int n_anc = 0, anc_blocks = 0;
    bool uploaded = false;              // descriptors already on their way to HBM (upload stream)
};

struct DlItem {
    int ue;
    int n_samples;
    const void* x;
    void* y;
    const void* taps;              // zero-copy snapshots or nullptr (ring)
};

struct UlCall {
    int cell;
    int n_samples;
    std::vector<int> ues;          // ascending
    std::vector<const void*> x;    // per ue (same order)
    std::vector<const void*> taps; // per ue: zero-copy snapshots or nullptr (ring)
    void* z;
    uint32_t flags;
    float2* partial = nullptr;     // group partials elsewhere than the cell's buffer (separate reduce pass)
};

// UL groups of one call: the UEs (ascending ids) partitioned by their
// outputs per lane (larger R first), ascending id inside each part, cut into
// groups of G consecutive UEs of one part; G is the tuned group size, raised
// until the cell has at most kMaxGroupsPerCell groups.  order: positions into
// the call's UE list; groups: [begin, end) ranges of order; R: per group.
struct UlPlan {
    std::vector<int> order;
    std::vector<std::pair<int, int>> groups;
    std::vector<int> R;
};

// Per-slot scratch of the slot builder, kept by the channel so that steady
// slots reuse its capacity instead of allocating.
struct SlotScratch {
    std::vector<int32_t> ns;
    std::vector<char> seen;
    std::vector<std::vector<int32_t>> ids;
    std::vector<std::vector<const void*>> xs, tps;
    std::vector<const DlItem*> order;
    using Key = std::tuple<int32_t, int32_t, int32_t, uintptr_t, int32_t, int32_t, int32_t>;
    std::vector<std::pair<Key, const DlItem*>> keyed;
    std::vector<ReduceDev> reds, reds_sep;
    std::vector<AnchorDev> ancs;
    std::vector<SelectDev> sels;
    std::vector<int> rs;
    UlPlan plan;
};

// Jobs and links of one launch class (accumulator rows) while a slot is built.
struct Cls {
    std::vector<LinkDev> links;
    std::vector<JobDev> jobs;
    std::vector<const Link*> lks;
};

}  // namespace

struct tt_channel {
    int device = 0;
    hipStream_t stream = nullptr;
    int iq_fmt = IQ_CI16;
    std::vector<tt_cell_cfg> cells;
    std::vector<int64_t> cell_clock;
    char* arena_base = nullptr;
    Arena arena;
    __half2* noise = nullptr;
    int64_t npool = 0;
    std::vector<Ue> ues;
    int active = 0;
    std::vector<float2*> cell_partial;  // [kMaxGroupsPerCell][n_ant][max_samples]
    std::vector<float2*> cell_acc;      // [n_ant][max_samples]
    std::vector<uint32_t*> cell_counters;  // per tile: UL groups finished (fused reduction)
    std::vector<DescBuf> desc;
    int desc_next = 0;
    unsigned long long* d_sat = nullptr;
    int64_t launches = 0, slots = 0;
    bool sticky = false;
    bool timing = false;
    int32_t timing_every = 1;   // time the slots whose launch index is a multiple of this
    int64_t timing_seq = 0;     // slots launched since timing was enabled
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    std::vector<int> ev_kind;  // per pending pair: 1 convolution kernel, 2 Jakes anchor pass, 0 whole graph
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
    double timed_ms[3] = {0.0, 0.0, 0.0};  // 0 every span, 1 the convolution kernel, 2 the anchor pass
    int64_t timed_launches[3] = {0, 0, 0};
    int tune_R = kDefaultR;
    int64_t tune_gen = 0;             // bumped by every set_tuning (link_r memos)
    int class_R[3][4][kMaxAnt] = {};  // outputs per lane per shape class (0: tune_R)
    int tune_G = kDefaultGroup;
    int tune_reduce = 2;  // 1 fused, 2 separate pass
    int tune_DG = kDefaultDlGroup;
    int tune_sub = 1;      // lane tiles per DL work item
    int tune_pf = 0;       // register prefetch of the next item (costs occupancy)
    int tune_persist = 0;  // workgroups per CU of a persistent grid; 0: one workgroup per tile
    int n_cu = 256;        // compute units of the device
    int tune_graph = 0;    // 1: slot kernels replayed from a captured hipGraph
    char* gdesc = nullptr; // fixed descriptor buffer read by the captured graph
    size_t gdesc_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream used only for capture
    hipStream_t up_stream = nullptr;   // uploads of staged slots' descriptors
    std::vector<int64_t> graph_sig;  // kernel arguments the graph was captured with
    int64_t graph_captures = 0, graph_launches = 0;
    hipEvent_t last_event = nullptr;  // completion of the last slot call
    int64_t desc_uses = 0;            // descriptor buffers taken so far
    struct PendingFree {
        hipEvent_t ev;
        int n;                          // arena blocks (a UE's state and its anchor tables)
        int64_t off[3], bytes[3];
    };
    std::vector<PendingFree> pending_free;  // released once the stream passes the event
    Cls slot_cls[kClasses];                 // slot-building scratch (capacity reused)
    SlotScratch scr;
    PreparedSlot prep;                      // a built slot awaiting its launch
    size_t desc_cap = 0;                    // bytes of every descriptor buffer, fixed at create
    std::vector<hipEvent_t> rel_free;       // events for deferred UE releases, created at create
};

namespace {

tt_status dev_fail(tt_channel* ch, hipError_t e, const char* what)
{
    if (ch)
        ch->sticky = true;
    return fail(TT_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void drop_graph(tt_channel* ch)
{
    if (ch->graph_exec)
        (void)hipGraphExecDestroy(ch->graph_exec);
    if (ch->graph)
        (void)hipGraphDestroy(ch->graph);
    ch->graph_exec = nullptr;
    ch->graph = nullptr;
    ch->graph_sig.clear();
}

// Adds the spans of every pending timing pair that has completed (or, with
// wait, of all of them) to the totals and returns the pairs to the pool.
hipError_t harvest_timing(tt_channel* ch, bool wait)
{
    size_t keep = 0;
    for (size_t i = 0; i < ch->ev_pending.size(); ++i) {
        const auto p = ch->ev_pending[i];
        const int kind = ch->ev_kind[i];
        hipError_t e = wait ? hipSuccess : hipEventQuery(p.second);
        if (e == hipErrorNotReady) {
            ch->ev_pending[keep] = p;
            ch->ev_kind[keep] = kind;
            ++keep;
            continue;
        }
        float t = 0.f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&t, p.first, p.second);
        if (e != hipSuccess)
            return e;
        ch->timed_ms[0] += t;
        ++ch->timed_launches[0];
        if (kind > 0) {
            ch->timed_ms[kind] += t;
            ++ch->timed_launches[kind];
        }
        ch->ev_free.push_back(p);
    }
    ch->ev_pending.resize(keep);
    ch->ev_kind.resize(keep);
    return hipSuccess;
}

// A timing pair from the pool created by tt_channel_enable_kernel_timing; when
// every pair is in flight, completed ones are harvested first.  If none is
// free the launch goes untimed (both events null): nothing is created here.
std::pair<hipEvent_t, hipEvent_t> take_event_pair(tt_channel* ch)
{
    std::pair<hipEvent_t, hipEvent_t> evp{nullptr, nullptr};
    if (ch->ev_free.empty())
        (void)harvest_timing(ch, false);
    if (!ch->ev_free.empty()) {
        evp = ch->ev_free.back();
        ch->ev_free.pop_back();
    }
    return evp;
}

#define TT_CHECK_STICKY(ch)                                                        \
    do {                                                                           \
        if (!(ch))                                                                 \
            return fail(TT_E_INVALID, "null channel");                             \
        if ((ch)->sticky)                                                          \
            return fail(TT_E_DEVICE, "channel is in a failed device state");       \
        hipError_t e_ = hipSetDevice((ch)->device);                                \
        if (e_ != hipSuccess)                                                      \
            return dev_fail((ch), e_, "hipSetDevice");                            \
    } while (0)

// Calls that change what a slot reads wait until a prepared slot is launched.
#define TT_CHECK_NO_PREPARED(ch)                                                   \
    do {                                                                           \
        if ((ch)->prep.valid)                                                      \
            return fail(TT_E_STATE, "a prepared slot waits for tt_channel_launch_prepared"); \
    } while (0)

template <class T>
T* at(tt_channel* ch, int64_t off) { return reinterpret_cast<T*>(ch->arena_base + off); }

// DL transmit streams: the serving cell's antennas, or with dl_tx_streams the
// stacked streams of several gNBs (serving cell first)
int link_tx(const tt_channel* ch, const tt_ue_cfg& c, int dir)
{
    if (dir == TT_DL)
        return c.dl_tx_streams > 0 ? c.dl_tx_streams : ch->cells[c.cell].n_ant;
    return c.n_tx;
}
int link_rx(const tt_channel* ch, const tt_ue_cfg& c, int dir) { return dir == TT_DL ? c.n_rx : ch->cells[c.cell].n_ant; }
int ring_cap_of(const tt_ue_cfg& c) { return c.ring_snapshots > 0 ? c.ring_snapshots : 512; }

// Sparse top-n selection entries one slot call of up to the cell's
// max_samples can need: snapshot blocks touched by N samples starting anywhere
// in a block, times antenna pairs, times the kept taps.
int64_t sel_entries(const tt_channel* ch, const tt_ue_cfg& c, int dir)
{
    if (c.mode == TT_TAPS_JAKES || c.sparse_taps <= 0 || c.sparse_taps >= c.n_taps)
        return 0;
    const int64_t P = c.snapshot_period, N = ch->cells[c.cell].max_samples;
    const int64_t blocks = (P - 1 + N - 1) / P + 1;
    return blocks * link_tx(ch, c, dir) * link_rx(ch, c, dir) * c.sparse_taps;
}

int64_t sel_bytes(const tt_channel* ch, const tt_ue_cfg& c, int dir)
{
    const int64_t e = sel_entries(ch, c, dir);
    return e ? align_up(e * (int64_t)sizeof(float4), kAlign) + align_up(e * 4, kAlign) : 0;
}

int64_t link_bytes(const tt_channel* ch, const tt_ue_cfg& c, int dir, int64_t* ring, int64_t* jakes, int64_t* hist)
{
    const int ntx = link_tx(ch, c, dir), nrx = link_rx(ch, c, dir);
    const int64_t per = (int64_t)nrx * ntx * c.n_taps;
    *ring = *jakes = 0;
    if (c.mode == TT_TAPS_JAKES)
        *jakes = align_up(per * kJakesPairs * (int64_t)kJakesPairBytes, kAlign);
    else
        *ring = align_up(per * ring_cap_of(c) * (c.tap_fmt == TT_TAP_F16 ? 4 : 8), kAlign);
    *hist = align_up((int64_t)ntx * kHist * 8, kAlign);
    return *ring + *jakes + *hist + sel_bytes(ch, c, dir);
}

int64_t ue_bytes(const tt_channel* ch, const tt_ue_cfg& c)
{
    int64_t a, b, h, tot = 0;
    for (int d = 0; d < 2; ++d)
        tot += link_bytes(ch, c, d, &a, &b, &h);
    return tot;
}

tt_status check_ue_cfg(const tt_channel* ch, const tt_ue_cfg* c)
{
    if (!c)
        return fail(TT_E_INVALID, "null ue cfg");
    if (c->cell < 0 || c->cell >= (int)ch->cells.size())
        return fail(TT_E_INVALID, "cell %d out of range", c->cell);
    if (c->n_taps < 1 || c->n_taps > TT_MAX_TAPS)
        return fail(TT_E_INVALID, "n_taps %d not in 1..%d", c->n_taps, TT_MAX_TAPS);
    if (c->n_tx < 1 || c->n_tx > TT_MAX_ANT || c->n_rx < 1 || c->n_rx > TT_MAX_ANT)
        return fail(TT_E_INVALID, "antenna counts must be 1..%d", TT_MAX_ANT);
    if (c->mode < TT_TAPS_HOLD || c->mode > TT_TAPS_JAKES)
        return fail(TT_E_INVALID, "bad tap mode %d", c->mode);
    if (c->mode != TT_TAPS_JAKES) {
        if (c->snapshot_period < 1 || c->snapshot_period > (1 << 30))
            return fail(TT_E_INVALID, "snapshot_period must be in 1..2^30");
        if (c->tap_fmt != TT_TAP_F32 && c->tap_fmt != TT_TAP_F16)
            return fail(TT_E_INVALID, "bad tap format");
        if (c->ring_snapshots < 0 || (c->ring_snapshots > 0 && c->ring_snapshots < 2))
            return fail(TT_E_INVALID, "ring_snapshots must be 0 or >= 2");
    }
    if (!(c->dl_sigma >= 0.0f))
        return fail(TT_E_INVALID, "dl_sigma must be >= 0");
    if (c->sparse_taps < 0)
        return fail(TT_E_INVALID, "sparse_taps must be >= 0");
    if (c->dl_tx_streams < 0 || c->dl_tx_streams > TT_MAX_ANT)
        return fail(TT_E_INVALID, "dl_tx_streams must be 0..%d", TT_MAX_ANT);
    if (c->dl_tx_streams > 0 && c->dl_tx_streams < ch->cells[c->cell].n_ant)
        return fail(TT_E_INVALID, "dl_tx_streams must include the serving cell's %d antennas",
                    ch->cells[c->cell].n_ant);
    if (c->sparse_taps > 0 && c->sparse_taps < c->n_taps && c->mode == TT_TAPS_JAKES)
        return fail(TT_E_INVALID, "sparse_taps applies to HOLD and LINEAR snapshots, not JAKES");
    return TT_OK;
}

// Bytes of every descriptor buffer, fixed at create: the largest slot table
// (each UE at most once per direction, so at most 2 max_ues links, each in
// its own job, selection and anchor entry at worst, one reduction per cell, and the
// alignment of every table), the largest batched ingest or resampling list
// (one entry per UE and direction) and the largest Jakes parameter set.
size_t desc_bytes_for(int max_ues, int n_cells)
{
    const size_t links = 2 * (size_t)max_ues;
    const size_t slot = links * (sizeof(LinkDev) + sizeof(JobDev) + sizeof(SelectDev) + sizeof(AnchorDev)) +
                        (size_t)n_cells * sizeof(ReduceDev) + (2 * kClasses + 7) * (size_t)kAlign;
    const size_t lists = links * std::max(sizeof(IngestDev), sizeof(ResampleDev));
    const size_t jakes = (size_t)TT_MAX_ANT * TT_MAX_ANT * TT_MAX_TAPS * kJakesPairs * kJakesPairBytes;
    return (size_t)align_up((int64_t)std::max({slot, lists, jakes, kDescMin}), 4096);
}

// Next descriptor buffer: waits until the GPU has consumed its last contents.
// Buffers are allocated at create with a capacity every call stays within,
// so nothing is allocated here.
tt_status take_desc(tt_channel* ch, size_t need, DescBuf** out)
{
    if (need > ch->desc_cap)
        return fail(TT_E_INVALID, "descriptor table of %zu bytes exceeds the %zu reserved at create", need,
                    ch->desc_cap);
    ++ch->desc_uses;
    DescBuf& d = ch->desc[ch->desc_next];
    ch->desc_next = (ch->desc_next + 1) % kDescBufs;
    if (d.pending) {
        hipError_t e = hipEventSynchronize(d.done);
        if (e != hipSuccess)
            return dev_fail(ch, e, "hipEventSynchronize");
        d.pending = false;
    }
    *out = &d;
    return TT_OK;
}

// ---------------------------------------------------------------------------
// Batching of one slot's work into launches
// ---------------------------------------------------------------------------

const UlPlan& ul_plan(tt_channel* ch, const std::vector<int>& ues);
int link_r(const tt_channel* ch, const Link& lk);


const UlPlan& ul_plan(tt_channel* ch, const std::vector<int>& ues)
{
    UlPlan& p = ch->scr.plan;
    const int U = (int)ues.size();
    std::vector<int>& rs = ch->scr.rs;
    rs.resize(U);
    for (int i = 0; i < U; ++i)
        rs[i] = link_r(ch, ch->ues[ues[i]].link[TT_UL]);
    p.order.resize(U);
    for (int i = 0; i < U; ++i)
        p.order[i] = i;
    if (!std::is_sorted(p.order.begin(), p.order.end(), [&](int a, int b) { return rs[a] > rs[b]; }))
        std::stable_sort(p.order.begin(), p.order.end(), [&](int a, int b) { return rs[a] > rs[b]; });
    int G = std::max(1, ch->tune_G);
    for (;;) {
        p.groups.clear();
        p.R.clear();
        for (int k = 0; k < U;) {
            int e = k;
            while (e < U && e - k < G && rs[p.order[e]] == rs[p.order[k]])
                ++e;
            p.groups.emplace_back(k, e);
            p.R.push_back(rs[p.order[k]]);
            k = e;
        }
        if ((int)p.groups.size() <= kMaxGroupsPerCell)
            break;
        ++G;
    }
    return p;
}

// Kernels work in the samples' storage units: int16 counts for ci16 (scale
// 2^12 per unit of amplitude), so noise scales are converted to those units.
float out_scale(const tt_channel* ch) { return ch->iq_fmt == IQ_CI16 ? 4096.0f : 1.0f; }

int nblocks_max(int mode, int period, int T)
{
    (void)mode;
    return (period - 1 + T - 1) / period + 1;
}

// Bytes of the raw copies the prefetching kernel streams into LDS for a link
// on items of `sub` lane tiles of kBlock * R outputs: the input words of
// every transmit stream (tile plus halo), and for dense HOLD/LINEAR
// snapshots the snapshots one tile's pairs are formed from (0 for the others).
int link_raw_x(const Link& lk, int R, int sub, int iq_fmt)
{
    const int Lp = (lk.L + R - 1) / R * R;
    const int HP = (Lp + 3) / 4 * 4;
    return lk.n_tx * (HP + kBlock * R * sub) * (iq_fmt == IQ_CI16 ? 4 : 8);
}

int link_raw_t(const Link& lk, int R, int sub)
{
    if (lk.nsel > 0)
        return 0;
    // Jakes links are read as LINEAR fp32 snapshots (their anchors)
    const int nb = nblocks_max(lk.mode, lk.period, kBlock * R * sub) + (lk.mode != M_HOLD ? 1 : 0);
    return nb * lk.n_rx * lk.n_tx * lk.L * (lk.tap_fmt == TAP_F16 ? 4 : 8);
}

int link_lds_calc(const Link& lk, int R, int sub)
{
    const int T = kBlock * R * sub;
    const int Lp = (lk.L + R - 1) / R * R;
    const int HP = (Lp + 3) / 4 * 4;
    const int nb = nblocks_max(lk.mode, lk.period, T);
    const int xs = lk.n_tx * R * ((HP + T) / R | 1) * 8;  // rows of odd length, as the kernel lays them out
    const int ts = nb * lk.n_rx * lk.n_tx * Lp * 16;
    // sparse top-n: strength and flag per staged tap, then the selected (H, D)
    // pairs and R staged-input offsets each
    const int ne = nb * lk.n_rx * lk.n_tx * Lp;
    const int sp = lk.nsel > 0 ? ((ne * 12 + 15) & ~15) + nb * lk.n_rx * lk.n_tx * lk.nsel * (16 + 4 * R) : 0;
    return xs + ts + sp;
}

int link_lds(const Link& lk, int R, int sub = 1)
{
    const int i = log2_r(R) + 4 * (sub == 1 ? 0 : sub == 2 ? 1 : 2);
    if (!lk.lds_memo[i])
        lk.lds_memo[i] = link_lds_calc(lk, R, sub);
    return lk.lds_memo[i];
}

// Lane tiles per DL item of a link at R outputs per lane: the channel's
// setting, halved until the item's staging fits the LDS budget; one tile
// with the LDS-copy prefetch or at R = 8 (the kernel has no such variant).
int link_sub(const tt_channel* ch, const Link& lk, int R)
{
    if (ch->tune_pf || R > 4)
        return 1;
    int sub = ch->tune_sub;
    while (sub > 1 && link_lds(lk, R, sub) > kLdsLimit)
        sub /= 2;
    return sub;
}

// Outputs per lane of a link for a call at its current clock: its shape
// class's schedule (or the channel's), halved until snapshot blocks and the
// clock sit on the lane grid and the tile's staging fits the LDS budget.  It
// depends on the link alone, never on the batch, and it does not change any
// output (the per-output arithmetic is the same for every R).
int link_r(const tt_channel* ch, const Link& lk)
{
    const int64_t key = ch->tune_gen * 8 + (lk.clock & 7);
    if (lk.r_key == key)
        return lk.r_memo;
    const int want = ch->class_R[lk.mode][taps_bucket(lk.L)][lk.n_rx - 1];
    int R = want ? want : ch->tune_R;
    while (R > 1 && ((lk.period & (R - 1)) != 0 || (lk.clock & (R - 1)) != 0 || link_lds(lk, R) > kLdsLimit))
        R /= 2;
    lk.r_key = key;
    lk.r_memo = R;
    return R;
}

tt_status check_taps_ready(tt_channel* ch, int ue, int dir, int n_samples)
{
    Link& lk = ch->ues[ue].link[dir];
    if (n_samples == 0)
        return TT_OK;
    if (lk.mode == M_JAKES) {
        if (!lk.jakes_set)
            return fail(TT_E_TAPS, "UE %d %s: Jakes parameters not set", ue, dir ? "UL" : "DL");
        return TT_OK;
    }
    const int64_t k_first = floor_div(lk.clock, lk.period);
    int64_t k_last = floor_div(lk.clock + n_samples - 1, lk.period);
    if (lk.mode == M_LINEAR)
        k_last += 1;
    if (k_first < lk.k_lo || k_last >= lk.k_hi)
        return fail(TT_E_TAPS, "UE %d %s: snapshots %lld..%lld needed, %lld..%lld set", ue, dir ? "UL" : "DL",
                    (long long)k_first, (long long)k_last, (long long)lk.k_lo, (long long)lk.k_hi - 1);
    return TT_OK;
}

LinkDev make_link_dev(tt_channel* ch, int ue, int dir, const void* x, const void* ext_taps)
{
    Link& lk = ch->ues[ue].link[dir];
    LinkDev d{};
    d.x = x;
    d.hist = at<float2>(ch, lk.hist_off);
    d.ring = lk.ring_off >= 0 ? at<void>(ch, lk.ring_off) : nullptr;
    d.k0 = floor_div(lk.clock, lk.period);
    d.r0 = (int32_t)(lk.clock - d.k0 * lk.period);
    d.ring_cap = lk.ring_cap;
    d.slot0 = lk.ring_cap ? (int32_t)(d.k0 - floor_div(d.k0, lk.ring_cap) * lk.ring_cap) : 0;
    if (ext_taps && lk.mode != M_JAKES) {
        d.ring = ext_taps;
        d.ring_cap = 0;
        d.kbase = d.k0;
    }
    d.period = lk.period;
    d.L = lk.L;
    d.n_tx = lk.n_tx;
    d.n_rx = lk.n_rx;
    d.mode = lk.mode;
    d.tap_fmt = lk.tap_fmt;
    if (lk.mode == M_JAKES) {
        // the convolution reads the call's anchors (written by the anchor
        // pass) as LINEAR fp32 snapshots kbase = k0, k0 + 1, ...
        d.ring = at<void>(ch, lk.anc_off);
        d.ring_cap = 0;
        d.slot0 = 0;
        d.kbase = d.k0;
        d.mode = M_LINEAR;
        d.tap_fmt = TAP_F32;
    }
    d.write_hist = 1;
    d.nsel = lk.nsel;
    return d;
}

// Runs one slot: DL items and UL calls, validated beforehand.
// Builds one slot (DL items and UL calls, validated beforehand): groups the
// work into jobs, stages the descriptor tables in pinned memory and advances
// the clocks.  Nothing is enqueued until launch_slot.
tt_status build_slot(tt_channel* ch, const std::vector<DlItem>& dl, const std::vector<UlCall>& ul)
{
    // Partition jobs by accumulator rows (n_rx of the link).
    // per-class scratch kept by the channel, so that steady slots reuse its capacity
    Cls (&cls)[kClasses] = ch->slot_cls;
    for (Cls& c : cls) {
        c.links.clear();
        c.jobs.clear();
        c.lks.clear();
    }
    std::vector<ReduceDev>& reds = ch->scr.reds;          // finished inside the FIR launch by the last group
    std::vector<ReduceDev>& reds_sep = ch->scr.reds_sep;  // finished by the reduce kernel (cells without UEs)
    reds.clear();
    reds_sep.clear();
    int red_max_n = 0, red_max_ant = 0;


    for (const UlCall& u : ul) {
        const tt_cell_cfg& cc = ch->cells[u.cell];
        const int U = (int)u.ues.size();
        if (U == 0 && !(u.flags & TT_UL_END) && !(u.flags & TT_UL_BEGIN))
            continue;
        const UlPlan& plan = ul_plan(ch, u.ues);
        const int ngroups = (int)plan.groups.size();
        float2* const pbase = u.partial ? u.partial : ch->cell_partial[u.cell];
        const bool fused = ch->tune_reduce == 1 && !u.partial;
        const bool direct = (u.flags & TT_UL_BEGIN) && (u.flags & TT_UL_END) && ngroups == 1;
        for (int g = 0; g < ngroups; ++g) {
            // the group's links go straight into its class's table
            Cls& kc = cls[class_of(cc.n_ant, plan.R[g])];
            const int link0 = (int)kc.links.size();
            for (int k = plan.groups[g].first; k < plan.groups[g].second; ++k) {
                const int i = plan.order[k];
                kc.links.push_back(make_link_dev(ch, u.ues[i], TT_UL, u.x[i], u.taps[i]));
                kc.lks.push_back(&ch->ues[u.ues[i]].link[TT_UL]);
            }
            JobDev j{};
            j.link0 = link0;
            j.nlinks = (int)kc.links.size() - link0;
            j.sub = 1;
            j.N = u.n_samples;
            j.n_out = cc.n_ant;
            j.red = -1;
            if (direct) {
                j.kind = J_FINAL;
                j.out = u.z;
                for (int r = 0; r < cc.n_ant; ++r)
                    j.noise_base[r] = mod_pool(cc.ul_noise_off[r] + ch->cell_clock[u.cell], ch->npool);
                j.sigma = cc.ul_sigma * out_scale(ch);
            } else {
                j.kind = J_PARTIAL;
                j.out = pbase + (int64_t)g * cc.n_ant * u.n_samples;
                j.red = fused ? (int)reds.size() : -1;
            }
            kc.jobs.push_back(j);
        }
        if (!direct) {
            ReduceDev rd{};
            rd.partial = pbase;
            rd.ngroups = ngroups;
            rd.N = u.n_samples;
            rd.n_ant = cc.n_ant;
            rd.stride = cc.max_samples;
            rd.acc = ch->cell_acc[u.cell];
            rd.z = u.z;
            for (int r = 0; r < cc.n_ant; ++r)
                rd.noise_base[r] = mod_pool(cc.ul_noise_off[r] + ch->cell_clock[u.cell], ch->npool);
            rd.sigma = cc.ul_sigma * out_scale(ch);
            rd.flags = (int)(u.flags & 3u);
            rd.counters = ch->cell_counters[u.cell];
            if (ngroups > 0 && fused) {
                reds.push_back(rd);
            } else {
                reds_sep.push_back(rd);
                red_max_n = std::max(red_max_n, u.n_samples);
                red_max_ant = std::max(red_max_ant, cc.n_ant);
            }
        }
    }
    std::vector<const DlItem*>& order = ch->scr.order;
    order.clear();
    for (const DlItem& d : dl)
        order.push_back(&d);

    // DL on the vector units: UEs grouped per workgroup; UEs reading the
    // same broadcast input with the same tap count share one staged input
    // tile.
    {
        using Key = SlotScratch::Key;
        auto& keyed = ch->scr.keyed;
        keyed.clear();
        for (const DlItem* d : order) {
            const Ue& u = ch->ues[d->ue];
            keyed.emplace_back(Key(u.cfg.n_rx, -link_r(ch, u.link[TT_DL]), d->n_samples, (uintptr_t)d->x, u.cfg.n_taps,
                                   u.link[TT_DL].n_tx, d->ue),
                               d);
        }
        // steady slots list their UEs in the same order: usually sorted already
        auto by_key = [](const std::pair<Key, const DlItem*>& a, const std::pair<Key, const DlItem*>& b) {
            return a.first < b.first;
        };
        if (!std::is_sorted(keyed.begin(), keyed.end(), by_key))
            std::sort(keyed.begin(), keyed.end(), by_key);
        for (size_t i = 0; i < keyed.size(); ++i)
            order[i] = keyed[i].second;
    }
    const int DG = std::max(1, ch->tune_DG);
    const float dl_scale = out_scale(ch);
    for (size_t i = 0; i < order.size();) {
        const Ue& u0 = ch->ues[order[i]->ue];
        const int R0 = link_r(ch, u0.link[TT_DL]);
        size_t j = i + 1;
        while (j < order.size() && (int)(j - i) < DG && ch->ues[order[j]->ue].cfg.n_rx == u0.cfg.n_rx &&
               order[j]->n_samples == order[i]->n_samples && link_r(ch, ch->ues[order[j]->ue].link[TT_DL]) == R0)
            ++j;
        // the group's links go straight into its class's table
        Cls& kc = cls[class_of(u0.cfg.n_rx, R0)];
        const int link0 = (int)kc.links.size();
        bool shared = true;
        int sub = ch->tune_sub;
        for (size_t k = i; k < j; ++k) {
            const DlItem& d = *order[k];
            const Ue& ue = ch->ues[d.ue];
            sub = std::min(sub, link_sub(ch, ue.link[TT_DL], R0));
            kc.links.push_back(make_link_dev(ch, d.ue, TT_DL, d.x, d.taps));
            LinkDev& ld = kc.links.back();
            ld.y = d.y;
            for (int r = 0; r < ue.cfg.n_rx; ++r)
                ld.noise_base[r] = mod_pool(ue.cfg.dl_noise_off[r] + ue.link[TT_DL].clock, ch->npool);
            ld.sigma = ue.cfg.dl_sigma * dl_scale;
            kc.lks.push_back(&ue.link[TT_DL]);
            shared = shared && d.x == order[i]->x && ue.cfg.n_taps == u0.cfg.n_taps &&
                     ue.link[TT_DL].n_tx == u0.link[TT_DL].n_tx;
        }
        JobDev jb{};
        jb.link0 = link0;
        jb.nlinks = (int)(j - i);
        jb.N = order[i]->n_samples;
        jb.n_out = u0.cfg.n_rx;
        jb.kind = J_DL;
        jb.red = -1;
        jb.shared_x = (shared && j - i > 1) ? 1 : 0;
        jb.sub = sub;
        kc.jobs.push_back(jb);
        i = j;
    }

    // Jakes links: one anchor pass per slot writes each call's anchors into
    // its link's table, [anchor][n_rx][n_tx][L] from anchor k0 on.
    std::vector<AnchorDev>& ancs = ch->scr.ancs;
    ancs.clear();
    int anc_blocks = 0;
    for (int c = 1; c < kClasses; ++c)
        for (const JobDev& j : cls[c].jobs)
            for (int i = 0; i < j.nlinks; ++i) {
                const Link& lk = *cls[c].lks[j.link0 + i];
                if (lk.mode != M_JAKES || j.N <= 0)
                    continue;
                const LinkDev& ld = cls[c].links[j.link0 + i];
                const int64_t count = (int64_t)(ld.r0 + j.N - 1) / ld.period + 2;
                if (count > lk.anc_cap || ld.k0 < 0)
                    return fail(TT_E_INVALID, "Jakes call of %d samples exceeds the cell's max_samples", j.N);
                AnchorDev a{};
                a.jakes = at<double>(ch, lk.jakes_off);
                a.out = at<float2>(ch, lk.anc_off);
                a.k0 = ld.k0;
                a.count = (int32_t)count;
                a.per = lk.per();
                a.K = ld.period;
                a.block0 = anc_blocks;
                ancs.push_back(a);
                const int64_t ngrp = (a.k0 + count - 1) / kAnchorGroup - a.k0 / kAnchorGroup + 1;
                anc_blocks += (int)((ngrp * a.per + kBlock - 1) / kBlock);
            }

    // Sparse links: one selection pass per slot writes every block's choice,
    // [block][n_rx][n_tx][nsel] per link from its first block on.
    std::vector<SelectDev>& sels = ch->scr.sels;
    sels.clear();
    int sel_blocks = 0;
    {
        auto blocks_of = [](const LinkDev& ld, int N) { return (int64_t)(ld.r0 + N - 1) / ld.period + 1; };
        for (int c = 1; c < kClasses; ++c)
            for (const JobDev& j : cls[c].jobs)
                for (int i = 0; i < j.nlinks; ++i) {
                    LinkDev& ld = cls[c].links[j.link0 + i];
                    if (ld.nsel == 0)
                        continue;
                    // each sparse link writes its selection into its own
                    // storage in the arena (sized at admission)
                    const Link& lk = *cls[c].lks[j.link0 + i];
                    const int64_t nb = blocks_of(ld, j.N);
                    const int groups = (int)nb * ld.n_rx * ld.n_tx;
                    if ((int64_t)groups * ld.nsel > lk.sel_cap)
                        return fail(TT_E_INVALID, "sparse call of %d samples exceeds the cell's max_samples", j.N);
                    float4* pairs = at<float4>(ch, lk.sel_off);
                    int32_t* delay = at<int32_t>(ch, lk.sel_off + align_up(lk.sel_cap * (int64_t)sizeof(float4), kAlign));
                    ld.spairs = pairs;
                    ld.sdelay = delay;
                    ld.sk0 = ld.k0;
                    SelectDev sd{};
                    sd.ring = ld.ring;
                    sd.ring_cap = ld.ring_cap;
                    sd.s0 = (int32_t)(ld.ring_cap ? ld.k0 - floor_div(ld.k0, ld.ring_cap) * ld.ring_cap
                                                  : ld.k0 - ld.kbase);
                    sd.period = ld.period;
                    sd.L = ld.L;
                    sd.n_rx = ld.n_rx;
                    sd.n_tx = ld.n_tx;
                    sd.tap_fmt = ld.tap_fmt;
                    sd.mode = ld.mode;
                    sd.nsel = ld.nsel;
                    sd.nblk = (int)nb;
                    sd.pairs = pairs;
                    sd.delay = delay;
                    sels.push_back(sd);
                    // blocks of the selection pass: groups of L rounded up to a power of two lanes
                    const int gl = ld.L <= 8 ? 8 : ld.L <= 16 ? 16 : ld.L <= 32 ? 32 : 64;
                    sel_blocks = std::max(sel_blocks, (groups * gl + kSelRounds * kBlock - 1) / (kSelRounds * kBlock));
                }
    }

    // Launch shapes per class.
    LaunchShape shape[kClasses];
    size_t need = 0;
    for (int c = 1; c < kClasses; ++c) {
        Cls& k = cls[c];
        if (k.jobs.empty())
            continue;
        // links of one shape share their LDS size: remember the last shape
        struct Shape {
            int L, n_tx, n_rx, mode, period, nsel, R, sub;
            bool operator==(const Shape& o) const {
                return L == o.L && n_tx == o.n_tx && n_rx == o.n_rx && mode == o.mode && period == o.period &&
                       nsel == o.nsel && R == o.R && sub == o.sub;
            }
        };
        Shape memo_key{-1, 0, 0, 0, 0, 0, 0, 0};
        int memo_lds = 0;
        auto lds_of = [&](const Link& lk, int R, int sub) {
            const Shape sk{lk.L, lk.n_tx, lk.n_rx, lk.mode, lk.period, lk.nsel, R, sub};
            if (!(sk == memo_key)) {
                memo_key = sk;
                memo_lds = link_lds(lk, R, sub);
            }
            return memo_lds;
        };
        // every link of the class runs at the class's R (link_r put it there),
        // on its job's tiles of kBlock * R * sub outputs
        const int R = class_r(c);
        int lds = 0, tiles = 0, uniform = -1;
        for (JobDev& j : k.jobs) {
            for (int i = 0; i < j.nlinks; ++i) {
                const int b = lds_of(*k.lks[j.link0 + i], R, j.sub);
                if (b > kLdsLimit)
                    return fail(TT_E_INVALID, "a link's taps do not fit the tile LDS budget (snapshot period or "
                                              "anchor spacing too small for its tap count and antennas)");
                lds = std::max(lds, b);
            }
            const int T = kBlock * R * j.sub;
            j.tile0 = tiles;
            j.ntiles = (j.N + T - 1) / T;
            tiles += j.ntiles;
            uniform = uniform == -1 ? j.ntiles : (uniform == j.ntiles ? uniform : 0);
        }
        int grid = tiles;
        if (ch->tune_persist > 0)
            grid = std::min(tiles, ch->tune_persist * ch->n_cu);
        // prefetch: room for the next item's raw copies after the staging
        // buffers, as far as the LDS budget allows (items that do not fit
        // are staged synchronously)
        int raw_off = (lds + 15) & ~15, rawx = 0, rawt = 0;
        if (ch->tune_pf) {
            for (const JobDev& j : k.jobs)
                for (int i = 0; i < j.nlinks; ++i) {
                    const Link& lk = *k.lks[j.link0 + i];
                    rawx = std::max(rawx, link_raw_x(lk, R, j.sub, ch->iq_fmt));
                    rawt = std::max(rawt, link_raw_t(lk, R, j.sub));
                }
            if (raw_off + rawx + rawt > kLdsLimit)
                rawt = 0;
            if (raw_off + rawx + rawt > kLdsLimit)
                rawx = 0;
        }
        const int total_lds = (rawx + rawt) > 0 ? raw_off + rawx + rawt : lds;
        int subt = 0;
        for (const JobDev& j : k.jobs)
            subt |= j.sub > 1 ? 1 : 0;
        shape[c] = LaunchShape{R, class_nrx(c), total_lds, tiles, grid, ch->tune_pf, std::max(uniform, 0), raw_off,
                               rawx, rawt, subt};
        need += k.links.size() * sizeof(LinkDev) + k.jobs.size() * sizeof(JobDev) + 2 * kAlign;
    }
    need += (reds.size() + reds_sep.size()) * sizeof(ReduceDev) + 2 * kAlign;
    need += sels.size() * sizeof(SelectDev) + kAlign;
    need += ancs.size() * sizeof(AnchorDev) + kAlign;

    DescBuf* db = nullptr;
    tt_status s = take_desc(ch, need, &db);
    if (s != TT_OK)
        return s;
    size_t off = 0;
    size_t link_off[kClasses], job_off[kClasses];
    for (int c = 1; c < kClasses; ++c) {
        Cls& k = cls[c];
        if (k.jobs.empty())
            continue;
        link_off[c] = off;
        std::memcpy(db->host + off, k.links.data(), k.links.size() * sizeof(LinkDev));
        off = align_up(off + k.links.size() * sizeof(LinkDev), kAlign);
        job_off[c] = off;
        std::memcpy(db->host + off, k.jobs.data(), k.jobs.size() * sizeof(JobDev));
        off = align_up(off + k.jobs.size() * sizeof(JobDev), kAlign);
    }
    const size_t red_off = off;
    if (!reds.empty()) {
        std::memcpy(db->host + off, reds.data(), reds.size() * sizeof(ReduceDev));
        off = align_up(off + reds.size() * sizeof(ReduceDev), kAlign);
    }
    const size_t red_sep_off = off;
    if (!reds_sep.empty()) {
        std::memcpy(db->host + off, reds_sep.data(), reds_sep.size() * sizeof(ReduceDev));
        off = align_up(off + reds_sep.size() * sizeof(ReduceDev), kAlign);
    }
    const size_t sel_off = off;
    if (!sels.empty()) {
        std::memcpy(db->host + off, sels.data(), sels.size() * sizeof(SelectDev));
        off = align_up(off + sels.size() * sizeof(SelectDev), kAlign);
    }
    const size_t anc_off = off;
    if (!ancs.empty()) {
        std::memcpy(db->host + off, ancs.data(), ancs.size() * sizeof(AnchorDev));
        off += ancs.size() * sizeof(AnchorDev);
    }
    PreparedSlot& P = ch->prep;
    P = PreparedSlot();
    P.valid = true;
    P.db = db;
    P.off = off;
    for (int c = 1; c < kClasses; ++c) {
        P.njobs[c] = (int)cls[c].jobs.size();
        if (P.njobs[c] == 0)
            continue;
        P.shape[c] = shape[c];
        P.link_off[c] = link_off[c];
        P.job_off[c] = job_off[c];
    }
    P.red_off = red_off;
    P.red_sep_off = red_sep_off;
    P.n_reds_sep = (int)reds_sep.size();
    P.red_max_n = red_max_n;
    P.red_max_ant = red_max_ant;
    P.sel_off = sel_off;
    P.n_sel = (int)sels.size();
    P.sel_blocks = sel_blocks;
    P.anc_off = anc_off;
    P.n_anc = (int)ancs.size();
    P.anc_blocks = anc_blocks;

    // Advance clocks.
    for (const DlItem& d : dl)
        ch->ues[d.ue].link[TT_DL].clock += d.n_samples;
    for (const UlCall& u : ul) {
        for (int ue : u.ues)
            ch->ues[ue].link[TT_UL].clock += u.n_samples;
        if (u.flags & TT_UL_END)
            ch->cell_clock[u.cell] += u.n_samples;
    }
    ++ch->slots;
    return TT_OK;
}

// Enqueues the prepared slot: descriptor upload, then its kernels (directly
// or as a replayed graph).
tt_status launch_slot(tt_channel* ch)
{
    PreparedSlot& P = ch->prep;
    DescBuf* db = P.db;
    const size_t off = P.off;
    tt_status s = TT_OK;
    hipError_t e;
    const bool graph = ch->tune_graph && off > 0;
    const bool timed = ch->timing && (ch->timing_seq++ % ch->timing_every) == 0;
    char* base = db->dev;
    if (graph) {
        // Replayed graphs read their descriptors from one fixed device buffer
        // (allocated at create with the descriptor capacity).
        base = ch->gdesc;
    }
    if (off > 0 && P.uploaded) {
        // staged: the upload was enqueued on the upload stream at prepare
        // time.  Once it has completed (the usual case: it ran beside the
        // previous slot) no wait is enqueued, so no barrier packet sits in
        // front of the slot's kernels.
        e = hipEventQuery(db->uploaded);
        if (e == hipErrorNotReady)
            e = hipStreamWaitEvent(ch->stream, db->uploaded, 0);
        if (e != hipSuccess)
            return dev_fail(ch, e, "upload wait");
    } else if (off > 0) {
        e = launch_copy(base, db->host_dev, (int64_t)off, ch->stream);
        if (e != hipSuccess)
            return dev_fail(ch, e, "descriptor upload");
        ++ch->launches;
    }
    // The slot's kernels; with `timed`, each convolution launch carries a pair
    // of HIP events stamped with that dispatch's own start and end times.
    auto enqueue = [&](bool timed, hipStream_t st) -> tt_status {
        if (P.n_anc > 0) {
            std::pair<hipEvent_t, hipEvent_t> evp{nullptr, nullptr};
            if (timed)
                evp = take_event_pair(ch);
            hipError_t ee = launch_anchor(reinterpret_cast<const AnchorDev*>(base + P.anc_off), P.n_anc,
                                          P.anc_blocks, st, evp.first, evp.second);
            if (ee != hipSuccess)
                return dev_fail(ch, ee, "Jakes anchor launch");
            if (timed && evp.first) {
                ch->ev_pending.push_back(evp);
                ch->ev_kind.push_back(2);
            }
            ++ch->launches;
        }
        if (P.n_sel > 0) {
            hipError_t ee = launch_select(reinterpret_cast<const SelectDev*>(base + P.sel_off), P.n_sel,
                                          P.sel_blocks, st);
            if (ee != hipSuccess)
                return dev_fail(ch, ee, "sparse selection launch");
            ++ch->launches;
        }
        for (int c = 1; c < kClasses; ++c) {
            if (P.njobs[c] == 0)
                continue;
            std::pair<hipEvent_t, hipEvent_t> evp{nullptr, nullptr};
            if (timed)
                evp = take_event_pair(ch);
            hipError_t ee = launch_fir(P.shape[c], reinterpret_cast<const JobDev*>(base + P.job_off[c]),
                                       P.njobs[c], reinterpret_cast<const LinkDev*>(base + P.link_off[c]),
                                       reinterpret_cast<const ReduceDev*>(base + P.red_off), ch->noise, ch->npool,
                                       ch->iq_fmt, ch->d_sat, st, evp.first, evp.second);
            if (ee != hipSuccess)
                return dev_fail(ch, ee, "convolution kernel launch");
            if (timed && evp.first) {
                ch->ev_pending.push_back(evp);
                ch->ev_kind.push_back(1);
            }
            ++ch->launches;
        }
        if (P.n_reds_sep > 0) {
            hipError_t ee = launch_reduce(reinterpret_cast<const ReduceDev*>(base + P.red_sep_off),
                                          P.n_reds_sep, P.red_max_n, P.red_max_ant, ch->noise, ch->npool,
                                          ch->iq_fmt, ch->d_sat, st);
            if (ee != hipSuccess)
                return dev_fail(ch, ee, "UL reduce launch");
            ++ch->launches;
        }
        return TT_OK;
    };
    if (!graph) {
        s = enqueue(timed, ch->stream);
        if (s != TT_OK)
            return s;
    } else {
        // Every kernel argument of the slot: a repeat replays the captured graph.
        std::vector<int64_t> sig;
        for (int c = 1; c < kClasses; ++c) {
            if (P.njobs[c] == 0)
                continue;
            const LaunchShape& h = P.shape[c];
            sig.insert(sig.end(), {c, h.R, h.nrx, h.lds_bytes, h.total_tiles, h.grid, h.prefetch, h.tiles_per_job,
                                   h.raw_off, h.rawx_bytes, h.rawt_bytes, h.subtiles, (int64_t)P.njobs[c],
                                   (int64_t)P.link_off[c], (int64_t)P.job_off[c]});
        }
        sig.insert(sig.end(), {(int64_t)P.red_off, (int64_t)P.red_sep_off, (int64_t)P.n_reds_sep, P.red_max_n,
                               P.red_max_ant, (int64_t)(uintptr_t)base,
                               (int64_t)P.sel_off, P.n_sel, P.sel_blocks, (int64_t)P.anc_off, P.n_anc,
                               P.anc_blocks});
        if (!ch->graph_exec || sig != ch->graph_sig) {
            if (ch->graph_exec) {
                // the previous graph may still be running: its exec is released after the stream passes it
                (void)hipStreamSynchronize(ch->stream);
                drop_graph(ch);
            }
            // captured on a private stream (the channel's may be the null
            // stream, which cannot be captured); replayed on the channel's
            if (!ch->cap_stream) {
                e = hipStreamCreateWithFlags(&ch->cap_stream, hipStreamNonBlocking);
                if (e != hipSuccess)
                    return dev_fail(ch, e, "capture stream");
            }
            e = hipStreamBeginCapture(ch->cap_stream, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess)
                return dev_fail(ch, e, "hipStreamBeginCapture");
            s = enqueue(false, ch->cap_stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(ch->cap_stream, &g);
            if (s != TT_OK)
                return s;
            if (e != hipSuccess)
                return dev_fail(ch, e, "hipStreamEndCapture");
            e = hipGraphInstantiate(&ch->graph_exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return dev_fail(ch, e, "hipGraphInstantiate");
            }
            ch->graph = g;
            ch->graph_sig = sig;
            ++ch->graph_captures;
        }
        std::pair<hipEvent_t, hipEvent_t> evp{nullptr, nullptr};
        if (timed) {
            evp = take_event_pair(ch);
            if (evp.first)
                (void)hipEventRecord(evp.first, ch->stream);
        }
        e = hipGraphLaunch(ch->graph_exec, ch->stream);
        if (e != hipSuccess)
            return dev_fail(ch, e, "hipGraphLaunch");
        if (timed && evp.first) {
            (void)hipEventRecord(evp.second, ch->stream);
            ch->ev_pending.push_back(evp);
            ch->ev_kind.push_back(0);
        }
        ++ch->graph_launches;
    }
    e = hipEventRecord(db->done, ch->stream);
    if (e != hipSuccess)
        return dev_fail(ch, e, "hipEventRecord");
    db->pending = true;
    ch->last_event = db->done;

    P.valid = false;
    return TT_OK;
}

// Runs one slot: build, then launch.
tt_status run_slot(tt_channel* ch, const std::vector<DlItem>& dl, const std::vector<UlCall>& ul)
{
    tt_status s = build_slot(ch, dl, ul);
    return s == TT_OK ? launch_slot(ch) : s;
}

// Work already enqueued may still read the blocks of `pf`: they go back to
// the arena once the stream passes this point.  The event comes from the
// pool created at create (max_ues events); if every one still guards a
// release, the oldest releases are waited for.
void reclaim(tt_channel* ch, bool wait);
tt_status defer_release(tt_channel* ch, tt_channel::PendingFree pf)
{
    if (ch->rel_free.empty())
        reclaim(ch, false);
    if (ch->rel_free.empty())
        reclaim(ch, true);
    if (ch->rel_free.empty())
        return fail(TT_E_STATE, "no release event available");
    hipEvent_t ev = ch->rel_free.back();
    hipError_t e = hipEventRecord(ev, ch->stream);
    if (e != hipSuccess)
        return dev_fail(ch, e, "release event");
    ch->rel_free.pop_back();
    pf.ev = ev;
    ch->pending_free.push_back(pf);
    return TT_OK;
}

// Returns pending UE memory to the arena once the GPU is past its last use;
// with wait = true it blocks until all pending releases are possible.
void reclaim(tt_channel* ch, bool wait)
{
    auto& v = ch->pending_free;
    for (size_t i = 0; i < v.size();) {
        hipError_t q = wait ? hipEventSynchronize(v[i].ev) : hipEventQuery(v[i].ev);
        if (q == hipSuccess) {
            for (int b = 0; b < v[i].n; ++b)
                ch->arena.release(v[i].off[b], v[i].bytes[b]);
            ch->rel_free.push_back(v[i].ev);
            v[i] = v.back();
            v.pop_back();
        } else {
            ++i;
        }
    }
}

tt_status check_ue_id(tt_channel* ch, int ue)
{
    if (ue < 0 || ue >= (int)ch->ues.size() || !ch->ues[ue].active)
        return fail(TT_E_INVALID, "unknown UE %d", ue);
    return TT_OK;
}

tt_status build_dl(tt_channel* ch, int32_t n, const int32_t* ue, const int32_t* n_samples, const void* const* x,
                   void* const* y, const void* const* taps, std::vector<DlItem>* out)
{
    if (n < 0)
        return fail(TT_E_INVALID, "negative UE count");
    if (n > 0 && (!ue || !n_samples || !x || !y))
        return fail(TT_E_INVALID, "null array argument");
    std::vector<char>& seen = ch->scr.seen;
    seen.assign(ch->ues.size(), 0);
    for (int i = 0; i < n; ++i) {
        tt_status s = check_ue_id(ch, ue[i]);
        if (s != TT_OK)
            return s;
        if (seen[ue[i]])
            return fail(TT_E_INVALID, "UE %d listed twice", ue[i]);
        seen[ue[i]] = 1;
        if (n_samples[i] < 0)
            return fail(TT_E_INVALID, "negative sample count");
        if (n_samples[i] > 0 && (!x[i] || !y[i]))
            return fail(TT_E_INVALID, "null IQ pointer for UE %d", ue[i]);
        // a sparse link's selection storage holds one call of up to the
        // cell's max_samples (sized at admission)
        const Link& dlk = ch->ues[ue[i]].link[TT_DL];
        if ((dlk.nsel > 0 || dlk.mode == M_JAKES) && n_samples[i] > ch->cells[ch->ues[ue[i]].cfg.cell].max_samples)
            return fail(TT_E_INVALID, "UE %d: a %s downlink call is limited to the cell's max_samples (%d)", ue[i],
                        dlk.nsel > 0 ? "sparse" : "Jakes", ch->cells[ch->ues[ue[i]].cfg.cell].max_samples);
        const void* ext = (taps && ch->ues[ue[i]].link[TT_DL].mode != M_JAKES) ? taps[i] : nullptr;
        if (!ext) {
            s = check_taps_ready(ch, ue[i], TT_DL, n_samples[i]);
            if (s != TT_OK)
                return s;
        }
        out->push_back(DlItem{ue[i], n_samples[i], x[i], y[i], ext});
    }
    // zero-length items do no work
    out->erase(std::remove_if(out->begin(), out->end(), [](const DlItem& d) { return d.n_samples == 0; }),
               out->end());
    return TT_OK;
}

tt_status build_ul(tt_channel* ch, int32_t cell, int32_t n_samples, int32_t n, const int32_t* ue,
                   const void* const* x, void* z, uint32_t flags, const void* const* taps, UlCall* out)
{
    if (cell < 0 || cell >= (int)ch->cells.size())
        return fail(TT_E_INVALID, "cell %d out of range", cell);
    if (n < 0 || n_samples < 0)
        return fail(TT_E_INVALID, "negative count");
    if (n_samples > ch->cells[cell].max_samples)
        return fail(TT_E_INVALID, "n_samples %d exceeds the cell's max_samples %d", n_samples,
                    ch->cells[cell].max_samples);
    if (flags & ~3u)
        return fail(TT_E_INVALID, "unknown UL flags");
    if (n > 0 && (!ue || !x))
        return fail(TT_E_INVALID, "null array argument");
    if ((flags & TT_UL_END) && n_samples > 0 && !z)
        return fail(TT_E_INVALID, "null UL output");
    struct Item {
        int ue;
        const void* x;
        const void* taps;
    };
    std::vector<Item> v;
    v.reserve(n);
    std::vector<char>& seen = ch->scr.seen;
    seen.assign(ch->ues.size(), 0);
    for (int i = 0; i < n; ++i) {
        tt_status s = check_ue_id(ch, ue[i]);
        if (s != TT_OK)
            return s;
        if (ch->ues[ue[i]].cfg.cell != cell)
            return fail(TT_E_INVALID, "UE %d is not in cell %d", ue[i], cell);
        if (seen[ue[i]])
            return fail(TT_E_INVALID, "UE %d listed twice", ue[i]);
        seen[ue[i]] = 1;
        if (n_samples > 0 && !x[i])
            return fail(TT_E_INVALID, "null IQ pointer for UE %d", ue[i]);
        const void* ext = (taps && ch->ues[ue[i]].link[TT_UL].mode != M_JAKES) ? taps[i] : nullptr;
        if (!ext) {
            s = check_taps_ready(ch, ue[i], TT_UL, n_samples);
            if (s != TT_OK)
                return s;
        }
        v.push_back(Item{ue[i], x[i], ext});
    }
    std::sort(v.begin(), v.end(), [](const Item& a, const Item& b) { return a.ue < b.ue; });
    out->cell = cell;
    out->n_samples = n_samples;
    out->flags = flags;
    out->z = z;
    for (auto& p : v) {
        out->ues.push_back(p.ue);
        out->x.push_back(p.x);
        out->taps.push_back(p.taps);
    }
    return TT_OK;
}

// UL with no UE: the output is the cell noise alone.  Handled by the reduce
// pass with zero groups (BEGIN clears, END adds noise).
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* tt_last_error(void) { return g_err.c_str(); }

tt_status tt_channel_create(const tt_channel_cfg* cfg, tt_channel** out)
{
    if (!cfg || !out)
        return fail(TT_E_INVALID, "null argument");
    *out = nullptr;
    if (cfg->max_ues < 1)
        return fail(TT_E_INVALID, "max_ues must be >= 1");
    if (cfg->n_cells < 1 || !cfg->cells)
        return fail(TT_E_INVALID, "need at least one cell");
    if (cfg->iq_fmt != TT_IQ_CI16 && cfg->iq_fmt != TT_IQ_CF32)
        return fail(TT_E_INVALID, "bad iq format");
    if (!cfg->noise_pool || cfg->noise_pool_len < 1)
        return fail(TT_E_INVALID, "noise pool required");
    if (cfg->noise_pool_len >= (int64_t)1 << 31)
        return fail(TT_E_INVALID, "noise pool longer than 2^31 - 1 samples");
    for (int c = 0; c < cfg->n_cells; ++c) {
        const tt_cell_cfg& cc = cfg->cells[c];
        if (cc.n_ant < 1 || cc.n_ant > TT_MAX_ANT)
            return fail(TT_E_INVALID, "cell %d: n_ant must be 1..%d", c, TT_MAX_ANT);
        if (cc.max_samples < 1)
            return fail(TT_E_INVALID, "cell %d: max_samples must be >= 1", c);
        if (!(cc.sample_rate_hz > 0))
            return fail(TT_E_INVALID, "cell %d: sample rate must be > 0", c);
        if (!(cc.ul_sigma >= 0.0f))
            return fail(TT_E_INVALID, "cell %d: ul_sigma must be >= 0", c);
    }
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess)
        return fail(TT_E_DEVICE, "hipSetDevice(%d): %s", cfg->device, hipGetErrorString(e));

    tt_channel* ch = new tt_channel();
    ch->device = cfg->device;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device) == hipSuccess && cus > 0)
            ch->n_cu = cus;
    }
    ch->stream = reinterpret_cast<hipStream_t>(cfg->hip_stream);
    ch->iq_fmt = cfg->iq_fmt;
    ch->cells.assign(cfg->cells, cfg->cells + cfg->n_cells);
    ch->cell_clock.assign(cfg->n_cells, 0);
    ch->ues.resize(cfg->max_ues);
    ch->npool = cfg->noise_pool_len;

    // Fixed state sizes, carved from the arena first.
    int64_t fixed = align_up(ch->npool * 4, kAlign);
    for (const tt_cell_cfg& cc : ch->cells) {
        fixed += align_up((int64_t)kMaxGroupsPerCell * cc.n_ant * cc.max_samples * 8, kAlign);
        fixed += align_up((int64_t)cc.n_ant * cc.max_samples * 8, kAlign);
        fixed += align_up(((int64_t)cc.max_samples + kBlock - 1) / kBlock * 4, kAlign);
    }
    if (cfg->hbm_budget_bytes < fixed) {
        delete ch;
        return fail(TT_E_NOMEM, "hbm_budget_bytes %lld below the fixed state %lld", (long long)cfg->hbm_budget_bytes,
                    (long long)fixed);
    }
    e = hipMalloc((void**)&ch->arena_base, cfg->hbm_budget_bytes);
    if (e != hipSuccess) {
        delete ch;
        return fail(TT_E_NOMEM, "arena of %lld bytes: %s", (long long)cfg->hbm_budget_bytes, hipGetErrorString(e));
    }
    ch->arena.init(cfg->hbm_budget_bytes);
    ch->noise = at<__half2>(ch, ch->arena.alloc(ch->npool * 4));
    for (const tt_cell_cfg& cc : ch->cells) {
        ch->cell_partial.push_back(
            at<float2>(ch, ch->arena.alloc((int64_t)kMaxGroupsPerCell * cc.n_ant * cc.max_samples * 8)));
        ch->cell_acc.push_back(at<float2>(ch, ch->arena.alloc((int64_t)cc.n_ant * cc.max_samples * 8)));
        const int64_t cb = ((int64_t)cc.max_samples + kBlock - 1) / kBlock * 4;
        ch->cell_counters.push_back(at<uint32_t>(ch, ch->arena.alloc(cb)));
    }
    e = hipMemcpy(ch->noise, cfg->noise_pool, ch->npool * 4, hipMemcpyHostToDevice);
    for (size_t c = 0; c < ch->cell_counters.size() && e == hipSuccess; ++c)
        e = hipMemset(ch->cell_counters[c], 0, ((int64_t)ch->cells[c].max_samples + kBlock - 1) / kBlock * 4);
    if (e == hipSuccess)
        e = hipMalloc((void**)&ch->d_sat, sizeof(unsigned long long));
    if (e == hipSuccess)
        e = hipMemset(ch->d_sat, 0, sizeof(unsigned long long));
    // Descriptor buffers (pinned host staging and device copies) and the
    // graph replay's fixed buffer, at the capacity every later call fits in,
    // and the events of deferred UE releases: the slot path allocates nothing.
    ch->desc_cap = desc_bytes_for(cfg->max_ues, cfg->n_cells);
    ch->desc.resize(kDescBufs);
    for (DescBuf& d : ch->desc) {
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&d.done, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&d.uploaded, hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&d.host, ch->desc_cap, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostGetDevicePointer((void**)&d.host_dev, d.host, 0);
        if (e == hipSuccess)
            e = hipMalloc((void**)&d.dev, ch->desc_cap);
        if (e == hipSuccess)
            d.cap = ch->desc_cap;
    }
    if (e == hipSuccess) {
        e = hipMalloc((void**)&ch->gdesc, ch->desc_cap);
        if (e == hipSuccess)
            ch->gdesc_cap = ch->desc_cap;
    }
    for (int i = 0; i < cfg->max_ues && e == hipSuccess; ++i) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess)
            ch->rel_free.push_back(ev);
    }
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&ch->up_stream, hipStreamNonBlocking);
    // the device's copy of the allocation-free call's scratch (resolved once per device)
    if (e == hipSuccess)
        e = noalloc_scratch_init(cfg->device);
    if (e != hipSuccess) {
        tt_channel_destroy(ch);
        return fail(TT_E_DEVICE, "create: %s", hipGetErrorString(e));
    }
    *out = ch;
    return TT_OK;
}

tt_status tt_channel_destroy(tt_channel* ch)
{
    if (!ch)
        return TT_OK;
    (void)hipSetDevice(ch->device);
    (void)hipStreamSynchronize(ch->stream);
    if (ch->up_stream)
        (void)hipStreamSynchronize(ch->up_stream);
    for (DescBuf& d : ch->desc) {
        if (d.host)
            (void)hipHostFree(d.host);
        if (d.dev)
            (void)hipFree(d.dev);
        if (d.done)
            (void)hipEventDestroy(d.done);
        if (d.uploaded)
            (void)hipEventDestroy(d.uploaded);
    }
    for (auto& p : ch->ev_pending) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    for (auto& p : ch->ev_free) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    for (auto& p : ch->pending_free)
        (void)hipEventDestroy(p.ev);
    drop_graph(ch);
    if (ch->cap_stream)
        (void)hipStreamDestroy(ch->cap_stream);
    if (ch->up_stream)
        (void)hipStreamDestroy(ch->up_stream);
    if (ch->gdesc)
        (void)hipFree(ch->gdesc);
    for (hipEvent_t ev : ch->rel_free)
        (void)hipEventDestroy(ev);
    if (ch->d_sat)
        (void)hipFree(ch->d_sat);
    if (ch->arena_base)
        (void)hipFree(ch->arena_base);
    delete ch;
    return TT_OK;
}

tt_status tt_channel_footprint(const tt_channel* ch, const tt_ue_cfg* ue, int64_t* bytes)
{
    if (!ch || !bytes)
        return fail(TT_E_INVALID, "null argument");
    tt_status s = check_ue_cfg(ch, ue);
    if (s != TT_OK)
        return s;
    *bytes = ue_bytes(ch, *ue);
    return TT_OK;
}

tt_status tt_channel_add_ue(tt_channel* ch, const tt_ue_cfg* cfg, int32_t* ue_id)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    if (!ue_id)
        return fail(TT_E_INVALID, "null ue_id");
    tt_status s = check_ue_cfg(ch, cfg);
    if (s != TT_OK)
        return s;
    int slot = -1;
    for (int i = 0; i < (int)ch->ues.size(); ++i)
        if (!ch->ues[i].active) {
            slot = i;
            break;
        }
    if (slot < 0)
        return fail(TT_E_ADMIT, "max_ues (%d) UEs already active", (int)ch->ues.size());
    const int64_t bytes = ue_bytes(ch, *cfg);
    reclaim(ch, false);
    int64_t off = ch->arena.alloc(bytes);
    if (off < 0 && !ch->pending_free.empty()) {
        reclaim(ch, true);
        off = ch->arena.alloc(bytes);
    }
    if (off < 0)
        return fail(TT_E_ADMIT, "UE footprint %lld bytes does not fit the arena (%lld of %lld used)",
                    (long long)bytes, (long long)ch->arena.used(), (long long)ch->arena.cap());
    Ue& u = ch->ues[slot];
    u = Ue();
    u.active = true;
    u.cfg = *cfg;
    u.off = off;
    u.bytes = bytes;
    u.m0 = ch->cell_clock[cfg->cell];
    int64_t p = off;
    for (int d = 0; d < 2; ++d) {
        Link& lk = u.link[d];
        int64_t rb, jb, hb;
        link_bytes(ch, *cfg, d, &rb, &jb, &hb);
        lk.L = cfg->n_taps;
        lk.n_tx = link_tx(ch, *cfg, d);
        lk.n_rx = link_rx(ch, *cfg, d);
        lk.mode = cfg->mode;
        lk.tap_fmt = cfg->mode == TT_TAPS_JAKES ? TAP_F32 : cfg->tap_fmt;
        lk.period = cfg->mode == TT_TAPS_JAKES ? 256 : cfg->snapshot_period;
        lk.ring_cap = cfg->mode == TT_TAPS_JAKES ? 0 : ring_cap_of(*cfg);
        lk.nsel = cfg->sparse_taps > 0 && cfg->sparse_taps < cfg->n_taps ? cfg->sparse_taps : 0;
        if (rb) {
            lk.ring_off = p;
            p += rb;
        }
        if (jb) {
            lk.jakes_off = p;
            p += jb;
        }
        lk.hist_off = p;
        p += hb;
        lk.sel_cap = sel_entries(ch, *cfg, d);
        if (lk.sel_cap > 0) {
            lk.sel_off = p;
            p += sel_bytes(ch, *cfg, d);
        }
    }
    hipError_t e = launch_zero(at<void>(ch, off), bytes, ch->stream);
    if (e != hipSuccess) {
        ch->arena.release(off, bytes);
        u = Ue();
        return dev_fail(ch, e, "zeroing UE state");
    }
    ++ch->active;
    *ue_id = slot;
    return TT_OK;
}

tt_status tt_channel_remove_ue(tt_channel* ch, int32_t ue)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    tt_status s = check_ue_id(ch, ue);
    if (s != TT_OK)
        return s;
    Ue& u = ch->ues[ue];
    tt_channel::PendingFree pf{};
    pf.off[pf.n] = u.off;
    pf.bytes[pf.n++] = u.bytes;
    for (const Link& lk : u.link)
        if (lk.anc_off >= 0) {
            pf.off[pf.n] = lk.anc_off;
            pf.bytes[pf.n++] = lk.anc_bytes;
        }
    s = defer_release(ch, pf);
    if (s != TT_OK)
        return s;
    u = Ue();
    --ch->active;
    return TT_OK;
}

static tt_status check_set_taps(tt_channel* ch, int32_t ue, int32_t dir, int64_t k0, int32_t count)
{
    tt_status s = check_ue_id(ch, ue);
    if (s != TT_OK)
        return s;
    if (dir != TT_DL && dir != TT_UL)
        return fail(TT_E_INVALID, "bad direction %d", dir);
    const Link& lk = ch->ues[ue].link[dir];
    if (lk.mode == M_JAKES)
        return fail(TT_E_STATE, "UE %d uses Jakes taps; use tt_channel_set_jakes", ue);
    if (k0 < 0 || count < 0)
        return fail(TT_E_INVALID, "negative snapshot index or count");
    if (count > lk.ring_cap)
        return fail(TT_E_INVALID, "count %d exceeds the ring capacity %d", count, lk.ring_cap);
    return TT_OK;
}

// Ring slot of snapshot k is k mod cap.  After writing [a, b) the valid
// window is the union with the old one, minus every old snapshot whose slot
// the write reused (those at distance >= cap from a written index).  A write
// that leaves a gap to the old window restarts it.
static void update_window(Link& lk, int64_t k0, int32_t count)
{
    if (count == 0)
        return;
    const int64_t a = k0, b = k0 + count, cap = lk.ring_cap;
    if (lk.k_hi <= lk.k_lo || a > lk.k_hi || b < lk.k_lo) {
        lk.k_lo = a;
        lk.k_hi = b;
        return;
    }
    lk.k_lo = std::max(std::min(lk.k_lo, a), b - cap);
    lk.k_hi = std::min(std::max(lk.k_hi, b), a + cap);
}

tt_status tt_channel_set_taps(tt_channel* ch, int32_t ue, int32_t dir, int64_t k0, int32_t count, const void* taps)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    tt_status s = check_set_taps(ch, ue, dir, k0, count);
    if (s != TT_OK)
        return s;
    if (count > 0 && !taps)
        return fail(TT_E_INVALID, "null taps");
    if (count == 0)
        return TT_OK;
    Link& lk = ch->ues[ue].link[dir];
    const int64_t per_bytes = (int64_t)lk.per() * lk.tap_bytes();
    // Copied into pinned staging before return, in chunks of whole snapshots
    // that fit one descriptor buffer; the uploads are stream-ordered.
    const int32_t chunk = (int32_t)std::max<int64_t>(1, (int64_t)ch->desc_cap / per_bytes);
    char* ring = at<char>(ch, lk.ring_off);
    const char* src = static_cast<const char*>(taps);
    for (int32_t c0 = 0; c0 < count; c0 += chunk) {
        const int32_t cn = std::min(chunk, count - c0);
        DescBuf* db = nullptr;
        s = take_desc(ch, (size_t)(cn * per_bytes), &db);
        if (s != TT_OK)
            return s;
        std::memcpy(db->host, src + c0 * per_bytes, (size_t)(cn * per_bytes));
        int32_t done = 0;
        hipError_t e = hipSuccess;
        while (done < cn && e == hipSuccess) {
            const int64_t slot = (k0 + c0 + done) % lk.ring_cap;
            const int32_t run = (int32_t)std::min<int64_t>(cn - done, lk.ring_cap - slot);
            e = hipMemcpyAsync(ring + slot * per_bytes, db->host + done * per_bytes, run * per_bytes,
                               hipMemcpyHostToDevice, ch->stream);
            done += run;
        }
        if (e == hipSuccess)
            e = hipEventRecord(db->done, ch->stream);
        if (e != hipSuccess)
            return dev_fail(ch, e, "tap upload");
        db->pending = true;
        ch->last_event = db->done;
    }
    update_window(lk, k0, count);
    return TT_OK;
}

tt_status tt_channel_set_taps_device(tt_channel* ch, int32_t n, const tt_taps_src* entries)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    if (n < 0 || (n > 0 && !entries))
        return fail(TT_E_INVALID, "bad entry list");
    std::vector<IngestDev> v;
    std::vector<char> seen(ch->ues.size() * 2, 0);
    int64_t max_taps = 0;
    for (int i = 0; i < n; ++i) {
        const tt_taps_src& en = entries[i];
        tt_status s = check_set_taps(ch, en.ue, en.dir, en.k0, en.count);
        if (s != TT_OK)
            return s;
        if (en.count > 0 && !en.src)
            return fail(TT_E_INVALID, "null source for entry %d", i);
        char& mark = seen[(size_t)en.ue * 2 + en.dir];
        if (mark)
            return fail(TT_E_INVALID, "UE %d direction %d listed twice", en.ue, en.dir);
        mark = 1;
        const Link& lk = ch->ues[en.ue].link[en.dir];
        if (en.count == 0)
            continue;
        IngestDev d{};
        d.src = en.src;
        d.ring = at<void>(ch, lk.ring_off);
        d.k0 = en.k0;
        d.count = en.count;
        d.cap = lk.ring_cap;
        d.per = lk.per();
        d.bytes_per_tap = lk.tap_bytes();
        v.push_back(d);
        max_taps = std::max<int64_t>(max_taps, (int64_t)d.count * d.per);
    }
    if (v.empty())
        return TT_OK;
    DescBuf* db = nullptr;
    tt_status s = take_desc(ch, v.size() * sizeof(IngestDev), &db);
    if (s != TT_OK)
        return s;
    std::memcpy(db->host, v.data(), v.size() * sizeof(IngestDev));
    hipError_t e = launch_copy(db->dev, db->host_dev, (int64_t)(v.size() * sizeof(IngestDev)), ch->stream);
    if (e == hipSuccess)
        e = launch_ingest(reinterpret_cast<const IngestDev*>(db->dev), (int)v.size(), max_taps, ch->stream);
    if (e == hipSuccess)
        e = hipEventRecord(db->done, ch->stream);
    if (e != hipSuccess)
        return dev_fail(ch, e, "tap ingest");
    db->pending = true;
    ch->last_event = db->done;
    ++ch->launches;
    for (int i = 0; i < n; ++i)
        if (entries[i].count > 0)
            update_window(ch->ues[entries[i].ue].link[entries[i].dir], entries[i].k0, entries[i].count);
    return TT_OK;
}

tt_status tt_channel_set_taps_cir(tt_channel* ch, int32_t n, const tt_cir_src* entries)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    if (n < 0 || (n > 0 && !entries))
        return fail(TT_E_INVALID, "bad entry list");
    std::vector<ResampleDev> v;
    std::vector<char> seen(ch->ues.size() * 2, 0);
    int max_count = 0;
    for (int i = 0; i < n; ++i) {
        const tt_cir_src& en = entries[i];
        tt_status s = check_set_taps(ch, en.ue, en.dir, en.k0, en.count);
        if (s != TT_OK)
            return s;
        if (en.n_paths < 0 || en.n_paths > TT_MAX_PATHS)
            return fail(TT_E_INVALID, "entry %d: n_paths must be 0..%d", i, TT_MAX_PATHS);
        if (!std::isfinite(en.t0_s))
            return fail(TT_E_INVALID, "entry %d: t0_s must be finite", i);
        if (en.count > 0 && en.n_paths > 0) {
            if (!en.delay_s || !en.gain)
                return fail(TT_E_INVALID, "null source for entry %d", i);
            if (((uintptr_t)en.delay_s | (uintptr_t)en.gain) % 8 != 0)
                return fail(TT_E_INVALID, "entry %d: sources must be 8-byte aligned", i);
        }
        char& mark = seen[(size_t)en.ue * 2 + en.dir];
        if (mark)
            return fail(TT_E_INVALID, "UE %d direction %d listed twice", en.ue, en.dir);
        mark = 1;
        const Link& lk = ch->ues[en.ue].link[en.dir];
        if (en.count == 0)
            continue;
        ResampleDev d{};
        d.delay = en.delay_s;
        d.gain = reinterpret_cast<const float2*>(en.gain);
        d.ring = at<void>(ch, lk.ring_off);
        d.k0 = en.k0;
        d.fs = ch->cells[ch->ues[en.ue].cfg.cell].sample_rate_hz;
        d.t0 = en.t0_s;
        d.count = en.count;
        d.cap = lk.ring_cap;
        d.n_paths = en.n_paths;
        d.n_rx = lk.n_rx;
        d.n_tx = lk.n_tx;
        d.L = lk.L;
        d.tap_fmt = lk.tap_fmt;
        v.push_back(d);
        max_count = std::max(max_count, en.count);
    }
    if (v.empty())
        return TT_OK;
    DescBuf* db = nullptr;
    tt_status s = take_desc(ch, v.size() * sizeof(ResampleDev), &db);
    if (s != TT_OK)
        return s;
    std::memcpy(db->host, v.data(), v.size() * sizeof(ResampleDev));
    hipError_t e = launch_copy(db->dev, db->host_dev, (int64_t)(v.size() * sizeof(ResampleDev)), ch->stream);
    if (e == hipSuccess)
        e = launch_resample(reinterpret_cast<const ResampleDev*>(db->dev), (int)v.size(), max_count, ch->stream);
    if (e == hipSuccess)
        e = hipEventRecord(db->done, ch->stream);
    if (e != hipSuccess)
        return dev_fail(ch, e, "CIR resampling");
    db->pending = true;
    ch->last_event = db->done;
    ++ch->launches;
    for (int i = 0; i < n; ++i)
        if (entries[i].count > 0)
            update_window(ch->ues[entries[i].ue].link[entries[i].dir], entries[i].k0, entries[i].count);
    return TT_OK;
}

tt_status tt_channel_set_jakes(tt_channel* ch, int32_t ue, int32_t dir, double doppler_hz, const double* pdp,
                               const double* theta, const double* phi)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    tt_status s = check_ue_id(ch, ue);
    if (s != TT_OK)
        return s;
    if (dir != TT_DL && dir != TT_UL)
        return fail(TT_E_INVALID, "bad direction %d", dir);
    Link& lk = ch->ues[ue].link[dir];
    if (lk.mode != M_JAKES)
        return fail(TT_E_STATE, "UE %d does not use Jakes taps", ue);
    if (!pdp || !theta || !phi)
        return fail(TT_E_INVALID, "null Jakes parameter array");
    if (!(doppler_hz >= 0.0) || !std::isfinite(doppler_hz))
        return fail(TT_E_INVALID, "doppler must be finite and >= 0");
    const double fs = ch->cells[ch->ues[ue].cfg.cell].sample_rate_hz;
    const double kPi = 3.14159265358979323846;
    // the parameter table, field by field: nu [8][per] (double), then a, b
    // and rot [8][per] (float2)
    const int per = lk.per();
    const size_t PP = (size_t)kJakesPairs * per;
    std::vector<double> nu(PP);
    std::vector<float2> ab(3 * PP);
    for (int rt = 0; rt < lk.n_rx * lk.n_tx; ++rt) {
        for (int l = 0; l < lk.L; ++l) {
            if (!(pdp[l] >= 0.0))
                return fail(TT_E_INVALID, "pdp must be >= 0");
            const double amp = std::sqrt(pdp[l] / 16.0);
            const double th = theta[(int64_t)rt * lk.L + l];
            const double* ph = phi + ((int64_t)rt * lk.L + l) * 16;
            for (int m = 0; m < kJakesPairs; ++m) {
                const size_t o = (size_t)m * per + (size_t)rt * lk.L + l;
                nu[o] = doppler_hz / fs * std::cos((2.0 * kPi * m + th) / 16.0);
                const double p0 = ph[m], p1 = ph[m + 8];
                ab[o] = make_float2((float)(amp * (std::cos(p0) + std::cos(p1))),
                                    (float)(amp * (std::sin(p0) + std::sin(p1))));
                ab[PP + o] = make_float2((float)(amp * (std::sin(p1) - std::sin(p0))),
                                         (float)(amp * (std::cos(p0) - std::cos(p1))));
            }
        }
    }
    // Anchor spacing: linear interpolation of exp(j w n) between anchors K
    // apart errs by at most (w K)^2 / 8 of the amplitude; keep it <= 1e-6.
    const double w = 2.0 * kPi * doppler_hz / fs;
    int K = 256;
    while (K > 1 && w * K * w * K / 8.0 > kJakesInterpBound)
        K /= 2;
    // one anchor step of each sinusoid pair, e^{j 2 pi nu K}, in FP64 rounded once
    for (size_t o = 0; o < PP; ++o) {
        double c = nu[o] * K;
        c -= std::floor(c);
        ab[2 * PP + o] = make_float2((float)std::cos(2.0 * kPi * c), (float)std::sin(2.0 * kPi * c));
    }
    // The link's anchor table: the anchors a call of up to the cell's
    // max_samples interpolates between, rewritten by each call's anchor
    // pass.  Allocated here (its size follows from K), kept while large
    // enough; a smaller one goes back to the arena once the stream is past it.
    const int64_t need = nblocks_max(M_LINEAR, K, ch->cells[ch->ues[ue].cfg.cell].max_samples) + 1;
    if (lk.anc_cap < need) {
        const int64_t bytes = need * lk.per() * 8;
        reclaim(ch, false);
        int64_t off = ch->arena.alloc(bytes);
        if (off < 0 && !ch->pending_free.empty()) {
            reclaim(ch, true);
            off = ch->arena.alloc(bytes);
        }
        if (off < 0)
            return fail(TT_E_ADMIT, "Jakes anchor table of %lld bytes does not fit the arena (%lld of %lld used)",
                        (long long)bytes, (long long)ch->arena.used(), (long long)ch->arena.cap());
        if (lk.anc_off >= 0) {
            tt_channel::PendingFree pf{};
            pf.off[0] = lk.anc_off;
            pf.bytes[0] = lk.anc_bytes;
            pf.n = 1;
            s = defer_release(ch, pf);
            if (s != TT_OK) {
                ch->arena.release(off, bytes);
                return s;
            }
        }
        lk.anc_off = off;
        lk.anc_cap = need;
        lk.anc_bytes = bytes;
    }
    DescBuf* db = nullptr;
    const size_t tbytes = PP * kJakesPairBytes;
    s = take_desc(ch, tbytes, &db);
    if (s != TT_OK)
        return s;
    std::memcpy(db->host, nu.data(), PP * sizeof(double));
    std::memcpy(db->host + PP * sizeof(double), ab.data(), 3 * PP * sizeof(float2));
    hipError_t e = hipMemcpyAsync(at<void>(ch, lk.jakes_off), db->host, tbytes,
                                  hipMemcpyHostToDevice, ch->stream);
    if (e == hipSuccess)
        e = hipEventRecord(db->done, ch->stream);
    if (e != hipSuccess)
        return dev_fail(ch, e, "Jakes parameter upload");
    db->pending = true;
    ch->last_event = db->done;
    lk.period = K;
    lk.forget_shape();
    lk.jakes_set = true;
    return TT_OK;
}

tt_status tt_channel_apply_dl(tt_channel* ch, int32_t n, const int32_t* ue, const int32_t* n_samples,
                              const void* const* x, void* const* y)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    std::vector<DlItem> dl;
    tt_status s = build_dl(ch, n, ue, n_samples, x, y, nullptr, &dl);
    if (s != TT_OK)
        return s;
    if (dl.empty())
        return TT_OK;
    return run_slot(ch, dl, {});
}

tt_status tt_channel_apply_ul(tt_channel* ch, int32_t cell, int32_t n_samples, int32_t n, const int32_t* ue,
                              const void* const* x, void* z, uint32_t flags)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    UlCall u;
    tt_status s = build_ul(ch, cell, n_samples, n, ue, x, z, flags, nullptr, &u);
    if (s != TT_OK)
        return s;
    if (n_samples == 0)
        return TT_OK;
    return run_slot(ch, {}, {u});
}

tt_status tt_channel_apply_ul_noalloc(tt_channel* ch, int32_t cell, int32_t n_samples, int32_t n,
                                      const int32_t* ue, const void* const* x, void* z, uint32_t flags)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    UlCall u;
    tt_status s = build_ul(ch, cell, n_samples, n, ue, x, z, flags, nullptr, &u);
    if (s != TT_OK)
        return s;
    if (n_samples == 0)
        return TT_OK;
    const int ngroups = (int)ul_plan(ch, u.ues).groups.size();
    const int64_t need = (int64_t)ngroups * ch->cells[cell].n_ant * n_samples * (int64_t)sizeof(float2);
    if (need > kNoallocScratchBytes)
        return fail(TT_E_INVALID, "UL partials of %lld bytes exceed the %lld-byte scratch of the allocation-free call",
                    (long long)need, (long long)kNoallocScratchBytes);
    void* p = noalloc_scratch(ch->device);
    if (!p)
        return fail(TT_E_STATE, "the device scratch was not resolved at create");
    u.partial = static_cast<float2*>(p);
    return run_slot(ch, {}, {u});
}

// Validates a slot description into DL items and UL calls.
static tt_status collect_slot(tt_channel* ch, const tt_slot* slot, std::vector<DlItem>& dl, std::vector<UlCall>& ul)
{
    if (!slot)
        return fail(TT_E_INVALID, "null slot");
    const int nc = (int)ch->cells.size();
    if ((slot->n_ul > 0 || slot->n_dl > 0) && !slot->cell_samples)
        return fail(TT_E_INVALID, "cell_samples required");
    if (slot->n_dl > 0) {
        std::vector<int32_t>& ns = ch->scr.ns;
        ns.resize(slot->n_dl);
        for (int i = 0; i < slot->n_dl; ++i) {
            if (!slot->dl_ue)
                return fail(TT_E_INVALID, "null dl_ue");
            const int u = slot->dl_ue[i];
            tt_status s = check_ue_id(ch, u);
            if (s != TT_OK)
                return s;
            ns[i] = slot->cell_samples[ch->ues[u].cfg.cell];
        }
        tt_status s = build_dl(ch, slot->n_dl, slot->dl_ue, ns.data(), slot->dl_x, slot->dl_y, slot->dl_taps, &dl);
        if (s != TT_OK)
            return s;
    }
    if (slot->n_ul > 0) {
        if (!slot->ul_ue || !slot->ul_x || !slot->ul_z)
            return fail(TT_E_INVALID, "null UL array");
        auto& ids = ch->scr.ids;
        auto& xs = ch->scr.xs;
        auto& tps = ch->scr.tps;
        ids.resize(nc);
        xs.resize(nc);
        tps.resize(nc);
        for (int c = 0; c < nc; ++c) {
            ids[c].clear();
            xs[c].clear();
            tps[c].clear();
        }
        for (int i = 0; i < slot->n_ul; ++i) {
            tt_status s = check_ue_id(ch, slot->ul_ue[i]);
            if (s != TT_OK)
                return s;
            const int c = ch->ues[slot->ul_ue[i]].cfg.cell;
            ids[c].push_back(slot->ul_ue[i]);
            xs[c].push_back(slot->ul_x[i]);
            tps[c].push_back(slot->ul_taps ? slot->ul_taps[i] : nullptr);
        }
        for (int c = 0; c < nc; ++c) {
            if (ids[c].empty() || slot->cell_samples[c] == 0)
                continue;
            UlCall u;
            tt_status s = build_ul(ch, c, slot->cell_samples[c], (int)ids[c].size(), ids[c].data(), xs[c].data(),
                                   slot->ul_z[c], TT_UL_BEGIN | TT_UL_END, slot->ul_taps ? tps[c].data() : nullptr,
                                   &u);
            if (s != TT_OK)
                return s;
            ul.push_back(std::move(u));
        }
    }
    return TT_OK;
}

tt_status tt_channel_apply_slot(tt_channel* ch, const tt_slot* slot)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    std::vector<DlItem> dl;
    std::vector<UlCall> ul;
    tt_status s = collect_slot(ch, slot, dl, ul);
    if (s != TT_OK || (dl.empty() && ul.empty()))
        return s;
    return run_slot(ch, dl, ul);
}

tt_status tt_channel_prepare_slot(tt_channel* ch, const tt_slot* slot)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    std::vector<DlItem> dl;
    std::vector<UlCall> ul;
    tt_status s = collect_slot(ch, slot, dl, ul);
    if (s != TT_OK)
        return s;
    if (dl.empty() && ul.empty()) {
        ch->prep = PreparedSlot();
        ch->prep.valid = true;  // nothing to enqueue
        return TT_OK;
    }
    s = build_slot(ch, dl, ul);
    if (s != TT_OK)
        return s;
    // Upload the descriptors now, on the upload stream, so that the copy
    // overlaps the slot in flight instead of preceding this one's kernels.
    // The buffer is free: taking it waited for its previous slot, which
    // waited for its own upload.  Graph replay reads one fixed buffer and
    // keeps the upload inside the launch.
    PreparedSlot& P = ch->prep;
    if (P.db && P.off > 0 && !ch->tune_graph) {
        hipError_t e = launch_copy(P.db->dev, P.db->host_dev, (int64_t)P.off, ch->up_stream);
        if (e == hipSuccess)
            e = hipEventRecord(P.db->uploaded, ch->up_stream);
        if (e != hipSuccess)
            return dev_fail(ch, e, "descriptor upload");
        ++ch->launches;
        P.uploaded = true;
    }
    return TT_OK;
}

tt_status tt_channel_launch_prepared(tt_channel* ch)
{
    TT_CHECK_STICKY(ch);
    if (!ch->prep.valid)
        return fail(TT_E_STATE, "no prepared slot");
    if (!ch->prep.db) {
        ch->prep.valid = false;
        return TT_OK;
    }
    return launch_slot(ch);
}

tt_status tt_channel_get_stats(tt_channel* ch, tt_stats* st)
{
    TT_CHECK_STICKY(ch);
    if (!st)
        return fail(TT_E_INVALID, "null stats");
    unsigned long long sat = 0;
    hipError_t e = hipStreamSynchronize(ch->stream);
    if (e == hipSuccess)
        e = hipMemcpy(&sat, ch->d_sat, sizeof sat, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return dev_fail(ch, e, "stats");
    reclaim(ch, true);
    st->saturated = (int64_t)sat;
    st->launches = ch->launches;
    st->slots = ch->slots;
    st->arena_bytes = ch->arena.cap();
    st->arena_used = ch->arena.used();
    st->active_ues = ch->active;
    st->graph_captures = ch->graph_captures;
    st->graph_launches = ch->graph_launches;
    return TT_OK;
}

tt_status tt_channel_sync(tt_channel* ch)
{
    TT_CHECK_STICKY(ch);
    hipError_t e = hipStreamSynchronize(ch->stream);
    if (e != hipSuccess)
        return dev_fail(ch, e, "hipStreamSynchronize");
    return TT_OK;
}

tt_status tt_channel_enable_kernel_timing(tt_channel* ch, int32_t on)
{
    TT_CHECK_STICKY(ch);
    if (on < 0)
        return fail(TT_E_INVALID, "timing period must be >= 0");
    double ms;
    int64_t n;
    tt_status s = tt_channel_kernel_time(ch, &ms, &n);
    if (s != TT_OK)
        return s;
    // the event pairs timed launches take, created here and not on the slot path
    while (on != 0 && (int)(ch->ev_free.size() + ch->ev_pending.size()) < kTimingPairs) {
        std::pair<hipEvent_t, hipEvent_t> p{nullptr, nullptr};
        hipError_t e = hipEventCreate(&p.first);
        if (e == hipSuccess)
            e = hipEventCreate(&p.second);
        if (e != hipSuccess) {
            if (p.first)
                (void)hipEventDestroy(p.first);
            return dev_fail(ch, e, "timing events");
        }
        ch->ev_free.push_back(p);
    }
    ch->timing = on != 0;
    ch->timing_every = on > 1 ? on : 1;
    ch->timing_seq = 0;
    for (int k = 0; k < 3; ++k) {
        ch->timed_ms[k] = 0.0;
        ch->timed_launches[k] = 0;
    }
    return TT_OK;
}

tt_status tt_channel_kernel_time_kind(tt_channel* ch, int32_t kind, double* ms, int64_t* launches)
{
    TT_CHECK_STICKY(ch);
    if (!ms || !launches || kind < 0 || kind > 2)
        return fail(TT_E_INVALID, "bad argument");
    hipError_t e = hipStreamSynchronize(ch->stream);
    if (e == hipSuccess)
        e = harvest_timing(ch, true);
    if (e != hipSuccess)
        return dev_fail(ch, e, "kernel timing");
    *ms = ch->timed_ms[kind];
    *launches = ch->timed_launches[kind];
    return TT_OK;
}

tt_status tt_channel_kernel_time(tt_channel* ch, double* ms, int64_t* launches)
{
    return tt_channel_kernel_time_kind(ch, 0, ms, launches);
}

tt_status tt_channel_set_tuning(tt_channel* ch, const tt_tuning* t)
{
    TT_CHECK_STICKY(ch);
    TT_CHECK_NO_PREPARED(ch);
    if (!t)
        return fail(TT_E_INVALID, "null tuning");
    const int R = t->outputs_per_lane;
    if (R != 0 && R != 1 && R != 2 && R != 4 && R != 8)
        return fail(TT_E_INVALID, "outputs_per_lane must be 0, 1, 2, 4 or 8");
    if (t->ul_group < 0)
        return fail(TT_E_INVALID, "ul_group must be >= 0");
    if (t->ul_reduce < 0 || t->ul_reduce > 2)
        return fail(TT_E_INVALID, "ul_reduce must be 0, 1 or 2");
    if (t->dl_subtiles != 0 && t->dl_subtiles != 1 && t->dl_subtiles != 2 && t->dl_subtiles != 4)
        return fail(TT_E_INVALID, "dl_subtiles must be 0, 1, 2 or 4");
    ch->tune_sub = t->dl_subtiles ? t->dl_subtiles : 1;
    ch->tune_R = R ? R : kDefaultR;
    ++ch->tune_gen;
    for (int m = 0; m < 3; ++m)
        for (int b = 0; b < 4; ++b)
            for (int r = 0; r < kMaxAnt; ++r) {
                const int v = t->outputs_by_class[m][b][r];
                if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8)
                    return fail(TT_E_INVALID, "outputs_by_class entries must be 0, 1, 2, 4 or 8");
            }
    std::memcpy(ch->class_R, t->outputs_by_class, sizeof ch->class_R);
    ch->tune_G = t->ul_group ? t->ul_group : kDefaultGroup;
    ch->tune_reduce = t->ul_reduce ? t->ul_reduce : 2;
    if (t->dl_group < 0)
        return fail(TT_E_INVALID, "dl_group must be >= 0");
    ch->tune_DG = t->dl_group ? t->dl_group : kDefaultDlGroup;
    if (t->prefetch < 0 || t->prefetch > 2)
        return fail(TT_E_INVALID, "prefetch must be 0, 1 or 2");
    ch->tune_pf = t->prefetch == 1 ? 1 : 0;
    if (t->persist < -1 || t->persist > 16)
        return fail(TT_E_INVALID, "persist must be -1 .. 16");
    if (t->graph < 0 || t->graph > 2)
        return fail(TT_E_INVALID, "graph must be 0, 1 or 2");
    ch->tune_graph = t->graph == 1 ? 1 : 0;
    ch->tune_persist = t->persist == 0 ? kDefaultPersist : (t->persist < 0 ? 0 : t->persist);
    return TT_OK;
}

}  // extern "C"

hipStream_t tt::channel_stream(tt_channel* ch) { return ch->stream; }
hipEvent_t tt::channel_last_event(tt_channel* ch) { return ch->last_event; }
int tt::channel_event_depth() { return kDescBufs; }
int64_t tt::channel_desc_uses(tt_channel* ch) { return ch->desc_uses; }
int tt::channel_iq_fmt(tt_channel* ch) { return ch->iq_fmt; }
const tt_cell_cfg* tt::channel_cells(tt_channel* ch, int* n)
{
    *n = (int)ch->cells.size();
    return ch->cells.data();
}
int tt::channel_device(tt_channel* ch) { return ch->device; }
const tt_ue_cfg* tt::channel_ue(tt_channel* ch, int ue)
{
    if (ue < 0 || ue >= (int)ch->ues.size() || !ch->ues[ue].active)
        return nullptr;
    return &ch->ues[ue].cfg;
}
void tt::set_error(const char* msg) { g_err = msg; }
