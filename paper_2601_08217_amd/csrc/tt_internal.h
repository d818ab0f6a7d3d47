// Internal declarations shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "tt_channel.h"

namespace tt {

constexpr int kBlock = 256;         // threads per workgroup (4 wave64)
constexpr int kMaxAnt = 4;
constexpr int kMaxTaps = 64;
constexpr int kHist = 64;           // history slots per (link, tx): >= kMaxTaps - 1
constexpr int kJakesPairs = 8;      // 16 sinusoids folded into 8 +-nu pairs
constexpr int64_t kNoallocScratchBytes = 16 << 20;  // device scratch of the allocation-free UL call

enum IqFmt : int32_t { IQ_CI16 = 0, IQ_CF32 = 1 };
enum TapFmt : int32_t { TAP_F32 = 0, TAP_F16 = 1 };
enum Mode : int32_t { M_HOLD = 0, M_LINEAR = 1, M_JAKES = 2 };
enum JobKind : int32_t { J_FINAL = 0, J_PARTIAL = 1, J_DL = 2 };

// Jakes parameters of one (rx, tx, tap): the 16 sinusoids come in pairs with
// opposite Doppler (nu_{m+8} = -nu_m), so h = sum_m c_m A_m + s_m B_m with
// (c_m, s_m) = (cos, sin)(2 pi nu_m n).  A link's table is stored field by
// field, each [kJakesPairs][per] over its per = n_rx n_tx L taps (so the
// lanes of a wave, on consecutive taps, read consecutive words):
//   nu  double  cycles per sample
//   a   float2  amp (e^{j phi_m} + e^{j phi_{m+8}})
//   b   float2  j amp (e^{j phi_m} - e^{j phi_{m+8}})
//   rot float2  (cos, sin)(2 pi nu K): one anchor step of K samples
constexpr int kJakesPairBytes = 32;
constexpr int kAnchorGroup = 8;     // Jakes anchors: one exact evaluation per group of this many

// One (UE, direction) link as seen by one launch.  Samples are used in their
// storage units (int16 counts for ci16, the float for cf32) from input to
// output; the host passes noise scales in the same units.
struct LinkDev {
    const void* x;            // [n_tx][N] input in the channel's iq format
    float2* hist;             // [n_tx][kHist] input units; hist[t][k] = x_t[n0 - (L-1) + k]
    const void* ring;         // HOLD/LINEAR taps: ring [R][n_rx][n_tx][L] (fp32 or fp16 complex),
                              // or, with ring_cap == 0, caller snapshots kbase, kbase + 1, ...
                              // (a Jakes link: its anchor table, as LINEAR fp32 snapshots)
    int64_t kbase;            // snapshot index of ring[0] when ring_cap == 0
    int64_t k0;               // floor(n0 / period): block of the call's first output
    int32_t r0;               // n0 - k0 * period
    int32_t ring_cap;         // R (snapshots); 0 = linear caller buffer
    int32_t slot0;            // ring slot of snapshot k0 (k0 mod ring_cap) when ring_cap > 0
    int32_t period;           // P (HOLD/LINEAR) or anchor spacing K (Jakes, seen as LINEAR)
    int32_t L, n_tx, n_rx;
    int32_t mode, tap_fmt;
    int32_t write_hist;       // 1: the tile at i = 0 rewrites the history
    // DL output of this link (J_DL jobs): y [n_rx][N]; noise index of output
    // i is (noise_base[r] + i) mod N_pool
    int32_t noise_base[kMaxAnt];
    void* y;
    float sigma;
    int32_t nsel;             // sparse top-n taps per snapshot block (0: every tap)
    // sparse: the selected (H, D) pairs and their delays, [block][n_rx][n_tx][nsel]
    // from snapshot block sk0 on (written by k_select before the convolution)
    const float4* spairs;
    const int32_t* sdelay;
    int64_t sk0;
};

// One Jakes link's anchors for one call (anchor pass).
struct AnchorDev {
    const double* jakes;      // the link's parameter table (nu, then a, b, rot)
    float2* out;              // [count][n_rx][n_tx][L]: anchors k0 .. k0 + count - 1
    int64_t k0;               // first anchor (>= 0)
    int32_t count;
    int32_t per;              // n_rx n_tx L
    int32_t K;                // anchor spacing (samples)
    int32_t block0;           // first workgroup of this entry (entries in order)
};

// One sparse link's snapshot blocks for the selection pass.
constexpr int kSelRounds = 4;       // group rounds per block of the selection pass

struct SelectDev {
    const void* ring;         // as LinkDev: ring (ring_cap > 0) or caller snapshots
    int32_t ring_cap;
    int32_t s0;               // snapshot index of the first block in ring (< ring_cap) or caller buffer
    int32_t period, L, n_rx, n_tx, tap_fmt, mode, nsel;
    int32_t nblk;             // blocks
    float4* pairs;            // [nblk][n_rx][n_tx][nsel]
    int32_t* delay;
};

// One piece of work of a launch over all its tiles: a DL group (links that
// each produce their own output, possibly sharing one broadcast input) or a
// UL group (links summed into one output).
struct JobDev {
    int32_t link0, nlinks;
    int32_t N;                // samples in this call
    int32_t tile0;            // first global tile index of this job
    int32_t ntiles;
    int32_t kind;             // J_DL (per-link outputs), J_FINAL (sum: noise + encode + store)
                              // or J_PARTIAL (sum: fp32 store)
    int32_t n_out;            // output antennas (rows of out)
    int32_t red;              // J_PARTIAL: index of the ReduceDev its last tile finishes, or -1
    void* out;                // J_FINAL: [n_out][N] iq format; J_PARTIAL: float2 [n_out][N]
    int32_t noise_base[kMaxAnt];  // J_FINAL: cell noise index of output 0 per antenna
    float sigma;
    int32_t shared_x;         // J_DL: every link reads the same input x
    int32_t sub;              // lane tiles per work item: a tile is kBlock * R * sub outputs,
                              // computed one lane tile after another (1 for UL jobs, whose
                              // accumulators carry across the links)
};

// UL second pass: z = (acc) + sum_g partial[g] (+ noise, encode).
struct ReduceDev {
    const float2* partial;    // [ngroups][n_ant][N]
    int32_t ngroups;
    int32_t N;
    int32_t n_ant;
    int32_t stride;           // samples per accumulator row
    float2* acc;              // cell accumulator [n_ant][stride]
    void* z;                  // [n_ant][N] iq format (END)
    int32_t noise_base[kMaxAnt];  // cell noise index of output 0 per antenna
    float sigma;
    int32_t flags;            // 1 BEGIN, 2 END
    uint32_t* counters;       // per tile: partial jobs finished (fused reduction), reset by the last
};

// Ring copy entry for the device tap ingest kernel.
struct IngestDev {
    const void* src;          // [count][per] complex (fp32 or fp16)
    void* ring;               // [cap][per]
    int64_t k0;
    int32_t count, cap;
    int32_t per;              // complex taps per snapshot (n_rx n_tx L)
    int32_t bytes_per_tap;    // 8 or 4
};

// One link's continuous-delay CIR steps for the resampling kernel.
struct ResampleDev {
    const double* delay;      // [count][n_paths] seconds
    const float2* gain;       // [count][n_paths][n_rx][n_tx]
    void* ring;               // [cap][n_rx][n_tx][L] in tap_fmt
    int64_t k0;               // snapshot index of step 0
    double fs;                // cell sample rate (Hz)
    double t0;                // delay of grid tap 0 (s)
    int32_t count, cap, n_paths;
    int32_t n_rx, n_tx, L;
    int32_t tap_fmt;
};

struct LaunchShape {
    int R;                    // outputs per lane
    int nrx;                  // accumulator rows (n_rx of every link of the launch)
    int lds_bytes;            // staging buffer
    int total_tiles;
    int grid;                 // workgroups (< total_tiles: persistent)
    int prefetch;             // 1: next item's raw input and taps copied into LDS while the current computes
    int tiles_per_job;        // > 0: every job has this many tiles (direct job lookup)
    int raw_off;              // prefetch: byte offset of the raw input words, then the raw tap words
    int rawx_bytes, rawt_bytes;  // prefetch: their sizes (0: that part is staged synchronously)
    int subtiles;             // 1: some job has items of several lane tiles (JobDev::sub > 1)
};

// kernels (tt_kernels.hip); ev0/ev1, when given, are stamped with the
// dispatch's own start and end times (kernel timing)
hipError_t launch_fir(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                      const ReduceDev* reds, const __half2* noise, int32_t npool, int iq_fmt,
                      unsigned long long* sat, hipStream_t st, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
// blocks: the workgroups of every entry (the last entry's block0 plus its own)
hipError_t launch_anchor(const AnchorDev* ent, int n, int blocks, hipStream_t st, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
// blocks: the largest over the entries of ceil(groups * select_lanes(L) / kBlock)
hipError_t launch_select(const SelectDev* ent, int n, int blocks, hipStream_t st);
hipError_t launch_reduce(const ReduceDev* red, int nred, int max_n, int max_ant,
                         const __half2* noise, int32_t npool, int iq_fmt,
                         unsigned long long* sat, hipStream_t st);
hipError_t launch_ingest(const IngestDev* ent, int n, int64_t max_taps, hipStream_t st);
// continuous-delay CIR resampling into tap rings (tt_resample.hip)
hipError_t launch_resample(const ResampleDev* ent, int n, int max_count, hipStream_t st);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);
// device scratch of the allocation-free UL call (tt_noalloc.hip): resolved once
// per device at channel create; the address, or nullptr before that
hipError_t noalloc_scratch_init(int device);
void* noalloc_scratch(int device);
hipError_t launch_copy(void* dst, const void* src, int64_t bytes, hipStream_t st);

}  // namespace tt

namespace tt {
// accessors used by the serving loop
hipStream_t channel_stream(tt_channel* ch);
// Event recorded at the end of the channel's last slot call; the channel
// re-records it channel_event_depth() calls later.
hipEvent_t channel_last_event(tt_channel* ch);
int channel_event_depth();
int64_t channel_desc_uses(tt_channel* ch);
int channel_iq_fmt(tt_channel* ch);
void set_error(const char* msg);
const tt_cell_cfg* channel_cells(tt_channel* ch, int* n);
int channel_device(tt_channel* ch);
// configuration of an active UE, or nullptr
const tt_ue_cfg* channel_ue(tt_channel* ch, int ue);



}  // namespace tt
