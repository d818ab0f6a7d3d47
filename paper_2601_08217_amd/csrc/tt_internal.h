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

enum IqFmt : int32_t { IQ_CI16 = 0, IQ_CF32 = 1 };
enum TapFmt : int32_t { TAP_F32 = 0, TAP_F16 = 1 };
enum Mode : int32_t { M_HOLD = 0, M_LINEAR = 1, M_JAKES = 2 };
enum JobKind : int32_t { J_FINAL = 0, J_PARTIAL = 1 };

// Jakes parameters of one (rx, tx, tap): the 16 sinusoids come in pairs with
// opposite Doppler (nu_{m+8} = -nu_m), so h = sum_m c_m A_m + s_m B_m with
// (c_m, s_m) = (cos, sin)(2 pi nu_m n).
struct JakesPair {
    double nu;        // cycles per sample
    float2 a;         // amp * (e^{j phi_m} + e^{j phi_{m+8}})
    float2 b;         // j * amp * (e^{j phi_m} - e^{j phi_{m+8}})
};
static_assert(sizeof(JakesPair) == 24, "JakesPair layout");

// One (UE, direction) link as seen by one launch.
struct LinkDev {
    const void* x;            // [n_tx][N] input in the channel's iq format
    float2* hist;             // [n_tx][kHist] cf32; hist[t][k] = x_t[n0 - (L-1) + k]
    const void* ring;         // HOLD/LINEAR tap ring [R][n_rx][n_tx][L] (fp32 or fp16 complex)
    const JakesPair* jakes;   // JAKES [n_rx][n_tx][L][kJakesPairs]
    int64_t n0;               // link sample clock at the first output of this call
    int32_t ring_cap;         // R (snapshots)
    int32_t period;           // P (HOLD/LINEAR) or anchor spacing K (JAKES)
    int32_t L, n_tx, n_rx;
    int32_t mode, tap_fmt;
    int32_t write_hist;       // 1: the tile at i = 0 rewrites the history
};

// One output of a launch: a DL UE (one link) or a UL group of links summed.
struct JobDev {
    int32_t link0, nlinks;
    int32_t N;                // samples in this call
    int32_t tile0;            // first global tile index of this job
    int32_t ntiles;
    int32_t kind;             // J_FINAL (noise + encode + store) or J_PARTIAL (fp32 store)
    int32_t n_out;            // output antennas (rows of out)
    int32_t pad0;
    void* out;                // J_FINAL: [n_out][N] iq format; J_PARTIAL: float2 [n_out][N]
    int64_t noise_n0;         // clock for the noise index
    int64_t noise_off[kMaxAnt];
    float sigma;
    int32_t pad1;
};

// UL second pass: z = (acc) + sum_g partial[g] (+ noise, encode).
struct ReduceDev {
    const float2* partial;    // [ngroups][n_ant][stride]
    int32_t ngroups;
    int32_t N;
    int32_t n_ant;
    int32_t stride;           // samples per partial row
    float2* acc;              // cell accumulator [n_ant][stride]
    void* z;                  // [n_ant][N] iq format (END)
    int64_t m0;               // cell clock (noise index)
    int64_t noise_off[kMaxAnt];
    float sigma;
    int32_t flags;            // 1 BEGIN, 2 END
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

struct LaunchShape {
    int R;                    // outputs per lane
    int nrx;                  // accumulator rows (max n_rx of the launch)
    int lds_bytes;
    int total_tiles;
};

// kernels (tt_kernels.hip)
hipError_t launch_fir(const LaunchShape& s, const JobDev* jobs, int njobs, const LinkDev* links,
                      const __half2* noise, int64_t npool, int iq_fmt,
                      unsigned long long* sat, hipStream_t st);
hipError_t launch_reduce(const ReduceDev* red, int nred, int max_n, int max_ant,
                         const __half2* noise, int64_t npool, int iq_fmt,
                         unsigned long long* sat, hipStream_t st);
hipError_t launch_ingest(const IngestDev* ent, int n, int64_t max_taps, hipStream_t st);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);

}  // namespace tt

namespace tt {
// accessors used by the serving loop
hipStream_t channel_stream(tt_channel* ch);
int channel_iq_fmt(tt_channel* ch);
void set_error(const char* msg);
const tt_cell_cfg* channel_cells(tt_channel* ch, int* n);

// LDS bytes a launch needs for tiles of T outputs.
int lds_bytes_for(int T, int Lp, int n_tx, int n_rx, int nblocks);

}  // namespace tt
