/*
 * tt_channel.h -- C ABI of the MI355X channel-emulation library.
 *
 * The library applies, per UE and per direction, a time-varying multi-tap
 * complex channel to baseband IQ streams on the GPU, keeping every UE's tap
 * state and sample history resident in device memory between slot calls.
 *
 * Operation (Tiny-Twin, Sec. III-B, the rfsim channel paragraph): every
 * receiver convolves the transmitted stream with its own time-varying channel
 * impulse response, y_u(t) = x(t) * h_u(t), a linear convolution that differs
 * per receiver.  Downlink: each UE receives the gNB's raw stream and applies
 * its own channel.  Uplink: the gNB convolves each UE's stream with that UE's
 * channel and sums the results.  Channels are complex taps on a fixed delay
 * grid, one snapshot per time step (Sec. IV, channel traces), or a Jakes
 * Doppler process (Sec. IV, 3GPP channels).  In discrete time, for receive
 * antenna r and UE sample clock n (n = 0 when the UE joins, inputs before it
 * are zero):
 *
 *   s_r[n] = sum_{t < n_tx} sum_{l < L} h_{r,t,l}[n] x_t[n - l]
 *   DL: y_r[n] = s_r[n] + dl_sigma * w[(dl_noise_off[r] + n) mod N_pool]
 *   UL: z_r[m] = sum_{UEs of the cell} s_{u,r}[m - m0_u]
 *                + ul_sigma * w[(ul_noise_off[r] + m) mod N_pool]
 *
 * with the tap indexed by OUTPUT time n; m is the cell's sample clock and m0_u
 * the cell sample at which UE u joined.  Tap modes (snapshot k = floor(n/P)):
 *   HOLD    h = H_k
 *   LINEAR  h = (1 - a) H_k + a H_{k+1},  a = (n mod P) / P
 *   JAKES   h = sqrt(p_l/16) sum_{m<16} exp(j(2 pi nu_m n + phi_m)),
 *           nu_m = (f_D / f_s) cos((2 pi m + theta) / 16)
 *           (the library evaluates JAKES exactly every K samples and
 *            interpolates linearly in between; K is chosen per link so that
 *            the interpolation error stays below 1e-6 of the tap amplitude)
 * w is a complex FP16 pool supplied at create.  ci16 samples are interleaved
 * int16 (I, Q) at scale 2^12: inputs decode exactly as I * 2^-12, outputs are
 * clamp(round_half_even(4096 v), -32768, 32767) per component.  Arithmetic is
 * FP32 with a fixed per-sample summation order (t, then l, ascending).
 *
 * Conventions shared by every call:
 *   - Status codes only; nothing throws across the ABI.  On failure the
 *     call has no side effects and tt_last_error() describes the cause.
 *   - A channel object is used from one host thread at a time.
 *   - All GPU work is enqueued on the channel's stream (cfg.hip_stream) and
 *     the calls return before it completes; results are ready when that
 *     stream reaches the point of the call (tt_channel_sync waits for it).
 *   - IQ buffers are DEVICE pointers owned by the caller; they must stay
 *     valid until the stream passes the call.  Tap, Jakes and noise inputs are
 *     HOST memory unless stated otherwise and are copied before the call
 *     returns.
 *   - Device errors (a failed launch or copy) are reported as TT_E_DEVICE and
 *     stay sticky: every later call returns TT_E_DEVICE.
 */
#ifndef TT_CHANNEL_H
#define TT_CHANNEL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TT_MAX_ANT 4    /* antennas per UE and per gNB */
#define TT_MAX_TAPS 64  /* taps per channel */

typedef struct tt_channel tt_channel; /* opaque, owned by the library */
typedef int32_t tt_status;

enum {
    TT_OK = 0,
    TT_E_INVALID = -1, /* bad argument, unknown UE, shape mismatch */
    TT_E_NOMEM = -2,   /* device or host allocation failed */
    TT_E_ADMIT = -3,   /* UE footprint does not fit the arena, or max_ues reached */
    TT_E_TAPS = -4,    /* taps needed by an apply call are not set */
    TT_E_DEVICE = -5,  /* HIP error (sticky) */
    TT_E_STATE = -6    /* call not valid in the current state */
};

enum { TT_DL = 0, TT_UL = 1 };
enum { TT_IQ_CI16 = 0, TT_IQ_CF32 = 1 };       /* interleaved I,Q */
enum { TT_TAP_F32 = 0, TT_TAP_F16 = 1 };       /* complex, interleaved re,im */
enum { TT_TAPS_HOLD = 0, TT_TAPS_LINEAR = 1, TT_TAPS_JAKES = 2 };
enum { TT_UL_BEGIN = 1, TT_UL_END = 2 };       /* tt_channel_apply_ul flags */

/* One cell: UEs of a cell share a sample rate; UL sums within a cell. */
typedef struct {
    double sample_rate_hz;                /* f_s, used by JAKES */
    int32_t n_ant;                        /* gNB antennas, 1..TT_MAX_ANT */
    int32_t max_samples;                  /* largest samples per slot call */
    float ul_sigma;                       /* UL noise std (complex) */
    int64_t ul_noise_off[TT_MAX_ANT];     /* UL noise pool offset per gNB antenna */
} tt_cell_cfg;

typedef struct {
    int32_t max_ues;                      /* UE slots */
    int64_t hbm_budget_bytes;             /* arena size; UEs are admitted by footprint */
    int32_t n_cells;
    const tt_cell_cfg *cells;             /* [n_cells], copied */
    int32_t iq_fmt;                       /* TT_IQ_CI16 or TT_IQ_CF32, inputs and outputs */
    const void *noise_pool;               /* host, complex FP16 [noise_pool_len][2], copied */
    int64_t noise_pool_len;               /* >= 1 */
    void *hip_stream;                     /* hipStream_t, or NULL for the null stream */
    int32_t device;                       /* HIP device ordinal */
} tt_channel_cfg;

typedef struct {
    int32_t cell;                         /* index into cfg.cells */
    int32_t n_taps;                       /* L, 1..TT_MAX_TAPS */
    int32_t n_tx, n_rx;                   /* UE antennas (UL transmit, DL receive) */
    int32_t mode;                         /* TT_TAPS_* */
    int32_t snapshot_period;              /* P in samples (HOLD, LINEAR) */
    int32_t tap_fmt;                      /* TT_TAP_F32 or TT_TAP_F16 (HOLD, LINEAR) */
    int32_t ring_snapshots;               /* tap-ring capacity per direction; 0 = default 512 */
    float dl_sigma;                       /* DL noise std (complex) */
    int64_t dl_noise_off[TT_MAX_ANT];     /* DL noise pool offset per UE antenna */
    int32_t dl_tx_streams;                /* 0: the DL input is the serving cell's n_ant
                                             streams.  > 0: the UE also hears other gNBs
                                             (inter-cell interference, Sec. V): its DL input
                                             stacks this many streams, the serving cell's
                                             first, all at the cell's sample rate, and its DL
                                             taps are [n_rx][dl_tx_streams][L]:
                                             y_r = sum over every stacked stream of h * x */
    int32_t sparse_taps;                  /* n > 0 (HOLD, LINEAR): per snapshot k and antenna
                                             pair, convolve only the n taps of largest
                                             |H_k|^2 (ties: smaller delay) over block k
                                             (Sec. III-C, sparse convolution); 0 or >= n_taps:
                                             every tap.  The selection storage (in the
                                             footprint) holds one call of up to the cell's
                                             max_samples, so a longer sparse downlink call
                                             is refused (TT_E_INVALID) */
} tt_ue_cfg;

/* Create a channel on cfg->device: allocates the arena (hbm_budget_bytes) and
 * copies the noise pool.  *out receives the handle.  TT_E_NOMEM if the arena
 * cannot be allocated or is smaller than the fixed state (noise pool, UL
 * scratch); TT_E_INVALID on a malformed cfg. */
tt_status tt_channel_create(const tt_channel_cfg *cfg, tt_channel **out);

/* Wait for the stream, free every device and host resource. NULL is a no-op. */
tt_status tt_channel_destroy(tt_channel *ch);

/* Device bytes a UE with this configuration occupies in the arena (tap rings
 * or Jakes parameters for both directions plus sample histories). */
tt_status tt_channel_footprint(const tt_channel *ch, const tt_ue_cfg *ue, int64_t *bytes);

/* Admit a UE: sub-allocates its footprint from the arena, zeroes its histories
 * and clocks (both start at 0), records the cell clock as its join point m0.
 * TT_E_ADMIT if the footprint does not fit or max_ues UEs are active. */
tt_status tt_channel_add_ue(tt_channel *ch, const tt_ue_cfg *ue, int32_t *ue_id);

/* Retire a UE at a slot boundary and return its memory to the arena. */
tt_status tt_channel_remove_ue(tt_channel *ch, int32_t ue_id);

/* Set tap snapshots k0 .. k0+count-1 of one direction (HOLD, LINEAR).
 * taps: HOST memory, layout [count][n_rx][n_tx][n_taps] complex in the UE's
 * tap_fmt; for TT_DL rx = UE antenna and tx = gNB antenna, for TT_UL rx = gNB
 * antenna and tx = UE antenna.  Snapshot k applies to UE-clock samples
 * [kP, (k+1)P) (LINEAR also interpolates toward k+1).  The ring keeps the
 * latest ring_snapshots snapshots; count must not exceed that.  Copied before
 * return. (Sec. IV: complex taps on a fixed delay grid, one per time step.) */
tt_status tt_channel_set_taps(tt_channel *ch, int32_t ue, int32_t dir, int64_t k0,
                              int32_t count, const void *taps);

/* Batched tap ingest from DEVICE memory: one kernel copies every entry into
 * its ring.  Same layout and rules as tt_channel_set_taps per entry.  The
 * sources must stay valid until the stream passes the call. */
typedef struct {
    int32_t ue, dir;
    int64_t k0;
    int32_t count;
    const void *src;                      /* device */
} tt_taps_src;
tt_status tt_channel_set_taps_device(tt_channel *ch, int32_t n, const tt_taps_src *entries);

/* Trace replay from continuous-delay CIRs (Sec. IV, channel traces: a
 * continuous CIR is resampled onto taps uniformly spaced in delay, one
 * snapshot per time step).  For each entry, time step s = 0 .. count-1 becomes
 * snapshot k0 + s of (ue, dir):
 *   H[r][t][l] = sum_p gain[s][p][r][t] * sinc(fs * (delay_s[s][p] - t0_s) - l)
 * for l = 0 .. n_taps-1, sinc(x) = sin(pi x)/(pi x), fs the cell's sample
 * rate: tap l sits at delay t0_s + l/fs, and a path off the grid leaks into
 * it through the truncated sinc.  Computed on the device in FP64 (four
 * contiguous quarters of the paths, each in index order, added in order) and
 * rounded once to the UE's tap_fmt, straight into the ring;
 * one kernel serves every entry.  delay_s: DEVICE FP64 [count][n_paths],
 * 8-byte aligned; gain: DEVICE complex FP32 (re, im) [count][n_paths][n_rx]
 * [n_tx] (rx/tx as in tt_channel_set_taps), 8-byte aligned; n_paths = 0 gives
 * zero taps.  Same ring and window rules as tt_channel_set_taps; JAKES links
 * are refused (TT_E_STATE).  The sources must stay valid until the stream
 * passes the call; non-finite delays or gains give non-finite taps. */
typedef struct {
    int32_t ue, dir;
    int64_t k0;
    int32_t count;                        /* time steps */
    int32_t n_paths;                      /* paths per step, 0 .. TT_MAX_PATHS */
    const double *delay_s;                /* device */
    const void *gain;                     /* device */
    double t0_s;                          /* delay of grid tap 0 (finite) */
} tt_cir_src;
#define TT_MAX_PATHS (1 << 20)
tt_status tt_channel_set_taps_cir(tt_channel *ch, int32_t n, const tt_cir_src *entries);

/* Jakes parameters of one direction (JAKES mode), HOST FP64 arrays:
 * pdp[n_taps] (tap powers p_l), theta[n_rx][n_tx][n_taps] (angle offsets),
 * phi[n_rx][n_tx][n_taps][16] (sinusoid phases).  f_s is the cell's rate.
 * The taps are evaluated at anchors K samples apart (K a power of two <= 256,
 * the largest whose linear interpolation errs by <= 1e-6 of the amplitude)
 * and interpolated linearly in between.  The first call (and any later one
 * that needs more anchors) allocates the direction's anchor table from the
 * arena: floor((K + max_samples - 2) / K) + 2 anchors (the cell's
 * max_samples) of n_rx * n_tx * n_taps * 8 bytes each, outside
 * tt_channel_footprint; TT_E_ADMIT if
 * it does not fit (nothing changed).  A Jakes downlink call is then limited
 * to the cell's max_samples (TT_E_INVALID).
 * (Sec. IV: time variation from a Jakes-based Doppler model.) */
tt_status tt_channel_set_jakes(tt_channel *ch, int32_t ue, int32_t dir, double doppler_hz,
                               const double *pdp, const double *theta, const double *phi);

/* Downlink for n UEs in one batched launch.  For UE ue[i]:
 * x[i] -> device [DL transmit streams][n_samples[i]] input, the cell's n_ant
 * streams or the UE's dl_tx_streams (pointers may alias: a
 * broadcast gNB stream), y[i] -> device [n_rx][n_samples[i]] output, in the
 * channel's iq_fmt.  Advances each UE's DL clock by n_samples[i].  A UE may
 * appear at most once.  n = 0 is a no-op. */
tt_status tt_channel_apply_dl(tt_channel *ch, int32_t n, const int32_t *ue,
                              const int32_t *n_samples, const void *const *x, void *const *y);

/* Uplink of n UEs of one cell, n_samples samples each.  x[i] -> device
 * [n_tx][n_samples] of UE ue[i].  Contributions are summed in ascending UE id
 * into the cell's FP32 accumulator: TT_UL_BEGIN clears it first, TT_UL_END
 * then adds the cell noise, writes z (device [n_ant][n_samples] in iq_fmt) and
 * advances the cell clock.  A batched call passes BEGIN|END; a per-UE
 * sequence passes BEGIN on the first call and END on the last, with the same
 * n_samples.  Every listed UE's UL clock advances by n_samples. */
tt_status tt_channel_apply_ul(tt_channel *ch, int32_t cell, int32_t n_samples, int32_t n,
                              const int32_t *ue, const void *const *x, void *z, uint32_t flags);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): tt_channel_apply_ul with
 * the same arguments and results, whose UL group partials live in a
 * library-wide device array of 16 MiB (one copy per device, held until the
 * process ends) instead of the channel's memory.  The call allocates no
 * device or pinned host memory (no hipMalloc, hipHostMalloc or hipFree);
 * the cross-group sum always runs as a separate reduction pass.  The
 * partials of a call, groups x the cell's antennas x n_samples x 8 bytes,
 * must fit the 16 MiB (else TT_E_INVALID, before any work); the groups are
 * those of apply_ul (the tuned ul_group, at most 64 per cell).  Every call on
 * one device shares that device's array: calls that overlap on one device
 * (other streams or channels) race and must not be issued. */
tt_status tt_channel_apply_ul_noalloc(tt_channel *ch, int32_t cell, int32_t n_samples, int32_t n,
                                      const int32_t *ue, const void *const *x, void *z, uint32_t flags);

/* DL and UL of one slot in a single batched launch sequence (what
 * apply_dl + apply_ul with BEGIN|END per cell compute, fused).  ul_z[c] is
 * the output of cell c (NULL when cell c has no UL UE in this slot);
 * cell_samples[c] is cell c's samples this slot.
 * Optional zero-copy taps (HOLD/LINEAR): dl_taps[i] / ul_taps[i], when the
 * array and the entry are non-NULL, is a DEVICE pointer to the snapshots this
 * call needs, consecutively in the UE's tap layout: snapshots k_first ..
 * k_last with k_first = floor(n0 / P), k_last = floor((n0 + N - 1) / P)
 * (+1 for LINEAR), n0 being the UE's clock in that direction.  They are read
 * by the kernels in place (no copy, the ring is not consulted) and must stay
 * valid and unchanged until the stream passes the call. */
typedef struct {
    int32_t n_dl;
    const int32_t *dl_ue;
    const void *const *dl_x;
    void *const *dl_y;
    int32_t n_ul;
    const int32_t *ul_ue;
    const void *const *ul_x;
    void *const *ul_z;                    /* [n_cells] */
    const int32_t *cell_samples;          /* [n_cells] */
    const void *const *dl_taps;           /* optional [n_dl], see above */
    const void *const *ul_taps;           /* optional [n_ul], see above */
} tt_slot;
tt_status tt_channel_apply_slot(tt_channel *ch, const tt_slot *slot);

/* tt_channel_apply_slot in two steps, for serving loops that build the next
 * slot while the current one runs.  prepare validates the slot exactly as
 * apply_slot does, builds its descriptor tables in pinned host memory and
 * advances the clocks, but enqueues nothing; launch_prepared then enqueues the
 * descriptor upload and the kernels.  The results equal apply_slot's.  While a
 * slot is prepared, every call that changes what a slot reads (UEs, taps,
 * Jakes parameters, tuning, other apply or prepare calls) fails with
 * TT_E_STATE, so the prepared tables stay valid; launch_prepared without a
 * prepared slot fails with TT_E_STATE too.  A prepared slot is dropped, not
 * run, if the channel is destroyed. */
tt_status tt_channel_prepare_slot(tt_channel *ch, const tt_slot *slot);
tt_status tt_channel_launch_prepared(tt_channel *ch);

/* Counters since create. */
typedef struct {
    int64_t saturated;                    /* ci16 output components clamped */
    int64_t launches;                     /* kernels launched directly or captured */
    int64_t slots;                        /* apply calls */
    int64_t arena_bytes, arena_used;
    int32_t active_ues;
    int64_t graph_captures;               /* hipGraph captures of a slot's kernels */
    int64_t graph_launches;               /* replays of a captured slot graph */
} tt_stats;
/* Reads device counters: waits for the stream. */
tt_status tt_channel_get_stats(tt_channel *ch, tt_stats *st);

/* Wait until all work enqueued on the channel's stream has completed. */
tt_status tt_channel_sync(tt_channel *ch);

/* Kernel timing: `on` = 0 turns it off; `on` = n >= 1 times every n-th slot
 * launched from now on (the first, then n later, ...; 1 times every slot).
 * In a timed slot every launch of a convolution kernel (and of the Jakes
 * anchor pass) on the channel's stream carries a pair of HIP events that the runtime stamps with that
 * dispatch's own start and end times (hipExtLaunchKernel), so a span is the
 * kernel's duration alone.  tt_channel_kernel_time returns the summed
 * milliseconds and launch count since enabling (waits).  Negative `on`:
 * TT_E_INVALID. */
tt_status tt_channel_enable_kernel_timing(tt_channel *ch, int32_t on);
tt_status tt_channel_kernel_time(tt_channel *ch, double *ms, int64_t *launches);
/* The same, per kernel kind: 0 every timed span, 1 the convolution kernel,
 * 2 the Jakes anchor pass.  With graph replay the spans cover whole graphs and count under kind 0
 * only.  Any other kind: TT_E_INVALID.  When every pre-created event pair is
 * in flight a launch goes untimed rather than creating events. */
tt_status tt_channel_kernel_time_kind(tt_channel *ch, int32_t kind, double *ms, int64_t *launches);

/* Launch schedule, chosen per workload shape by the project's autotuner.
 * Every field 0 means the library default.  None of them changes results
 * except ul_group and ul_reduce, which change the UL summation order within
 * the FP32 tolerance (DL outputs are bit-identical under every setting).
 * While a slot is prepared the call fails with TT_E_STATE. */
typedef struct {
    int32_t outputs_per_lane;             /* consecutive outputs per lane R: 1, 2, 4 or 8 */
    int32_t ul_group;                     /* UEs accumulated per UL workgroup, >= 1 */
    int32_t ul_reduce;                    /* 1: cross-group UL sum fused into the convolution
                                             launch (last group of a tile finishes it);
                                             2: separate reduction pass */
    int32_t dl_group;                     /* DL UEs processed per workgroup (sharing one staged
                                             input when they read the same broadcast stream) */
    int32_t prefetch;                     /* 1: copy the next item's raw input and tap
                                             snapshots from memory straight into LDS
                                             (global_load_lds) while the current one
                                             computes, then unpack them after its
                                             barrier; 2: stage each item after the
                                             previous one (default) */
    int32_t persist;                      /* > 0: persistent grid of this many workgroups per
                                             compute unit, each working through a strided list
                                             of tiles; -1: one workgroup per tile */
    int32_t graph;                        /* 1: the slot's kernels are captured once into a
                                             hipGraph and replayed while their launch
                                             arguments repeat (re-captured when the batch
                                             shape changes); 2: direct launches (default).
                                             With kernel timing on, the events bracket the
                                             whole replayed graph */
    int32_t outputs_by_class[3][4][TT_MAX_ANT];
                                          /* outputs per lane of links of one shape class,
                                             [tap mode][taps <= 8, <= 16, <= 32, <= 64]
                                             [receive antennas - 1] (1, 2, 4 or 8; 0: use
                                             outputs_per_lane).  A slot runs one convolution
                                             launch per (receive antennas, outputs per lane)
                                             with work; UL groups hold UEs of one class */
    int32_t dl_subtiles;                  /* lane tiles per DL work item: 1, 2 or 4.  A DL
                                             item (one UE over one tile) stages its input and
                                             taps once for this many tiles of 256 * R outputs
                                             and computes them one after another, spreading
                                             the per-item staging and barriers; lowered for
                                             a link whose staging would not fit the LDS
                                             budget.  One tile with prefetch = 1 or at 8
                                             outputs per lane, and for UL items (their sums
                                             are held across the group's UEs) */
} tt_tuning;
tt_status tt_channel_set_tuning(tt_channel *ch, const tt_tuning *tuning);

/* ---------------------------------------------------------------------------
 * Serving loop (slot-paced continuous batching).
 *
 * Each slot tick: retire UEs whose session ended, admit queued joins in
 * arrival order while the concurrent-UE cap and the arena (HBM footprint)
 * allow (a join that does not fit waits at the head of the queue), ingest
 * the next tap snapshots of every active UE from its device-resident pool,
 * then run DL and UL of all active UEs in one batched call (or, with
 * `plain`, one call per UE and direction).  Latency of a slot is host time
 * to the completion of its GPU work from its tick when paced (slot_us > 0,
 * so a launch held back past the tick counts against the budget), else from
 * the start of its submission.
 * (Tiny-Twin, Sec. III-A: compute-time fidelity and multi-user scalability
 * of slot execution; Sec. III-C: per-UE parallel convolution.)
 * ------------------------------------------------------------------------- */
typedef struct {
    tt_ue_cfg cfg;                 /* channel configuration of the UE */
    int64_t arrive_slot;           /* slot at which the join request arrives */
    int64_t session_slots;         /* slots served after admission; <= 0: to the end */
    const void *ul_x;              /* device [x_slots][n_tx][N_cell]: UL input of the
                                      UE's j-th served slot is block j mod x_slots */
    int32_t x_slots;
    const void *taps[2];           /* HOLD/LINEAR, device, per direction:
                                      [tap_len + 1][n_rx][n_tx][L] in tap_fmt; snapshot
                                      k is entry k mod tap_len (entry tap_len repeats
                                      entry 0 so that runs need not wrap) */
    int64_t tap_len;
    double doppler_hz[2];          /* JAKES, per direction: host parameters as in */
    const double *pdp[2];          /* tt_channel_set_jakes, applied at admission  */
    const double *theta[2];
    const double *phi[2];
    void *dl_y;                    /* device [y_slots][n_rx][N_cell]: DL output of
                                      cell slot s goes to block s mod y_slots */
    int32_t y_slots;
} tt_stream;

typedef struct {
    int32_t n_slots;               /* capacity of the per-slot record arrays (total slots run) */
    double slot_us;                /* > 0: slots start on ticks slot_us apart; 0: back to back */
    int32_t max_active;            /* concurrent-UE cap (<= max_ues) */
    const void *const *dl_x;       /* per cell, device [x_slots][n_ant][N]: block s mod x_slots */
    int32_t x_slots;
    void *const *ul_z;             /* per cell, device [z_slots][n_ant][N]: block s mod z_slots */
    int32_t z_slots;
    const int32_t *cell_samples;   /* per cell: samples per slot */
    int32_t plain;                 /* 1: one call per UE and direction, no batching */
    int32_t copy_taps;             /* 1: always copy snapshots into the tap rings; 0: hand
                                      the kernels zero-copy pointers into the pools when
                                      the slot's snapshots are contiguous there */
    double *lat_us;                /* optional [n_slots]: per-slot latency */
    int32_t *active;               /* optional [n_slots]: active UEs per slot */
    int64_t *admit_slot;           /* optional [n_streams]: admission slot or -1 */
    int64_t *leave_slot;           /* optional [n_streams]: slot of retirement or -1 */
} tt_serve_cfg;

typedef struct {
    int64_t slots, link_samples, ue_slots;
    double wall_s;                 /* first submission to last completion */
    double lat_p50_us, lat_p99_us, lat_max_us, lat_mean_us;
    double lat_p99_full_us;        /* p99 over slots with max_active UEs active */
    int64_t full_slots, misses;    /* misses: latency > slot budget (slot_us, or 500) */
    int64_t admitted, left, queued_end, max_queue;
    int32_t max_active, min_active;
    double host_us_mean;           /* host time per slot spent submitting its work */
    int64_t late_starts;           /* paced: slots launched more than slot_us / 10 after their tick */
    double start_lag_max_us;       /* paced: largest delay from a tick to its slot's launch */
    double build_us_mean;          /* host time per slot building it (ahead of its launch) */
    double window_wait_us_mean;    /* host time per slot blocked on the in-flight window */
} tt_serve_stats;

typedef struct tt_server tt_server;

/* A serving loop over a channel and a fixed set of streams (copied; the
 * device sources and the optional record arrays must outlive the server).
 * Slot indices count from 0 over all tt_server_run calls.  Every UE hears its
 * cell's DL stream: a stream with dl_tx_streams != 0 is refused
 * (TT_E_INVALID). */
tt_status tt_server_create(tt_channel *ch, const tt_serve_cfg *cfg, int32_t n_streams, const tt_stream *streams,
                           tt_server **out);

/* Runs the next n_slots slots (pacing, if any, restarts at the call) and
 * waits for their GPU work.  Fails with TT_E_INVALID past cfg->n_slots. */
tt_status tt_server_run(tt_server *srv, int32_t n_slots);

/* Statistics over the slots run since the last reset (reset != 0 clears). */
tt_status tt_server_stats(tt_server *srv, tt_serve_stats *stats, int32_t reset);

/* Retires every active UE and frees the server. NULL is a no-op. */
tt_status tt_server_destroy(tt_server *srv);

/* One-shot: create, run cfg->n_slots slots, report, destroy. */
tt_status tt_serve(tt_channel *ch, const tt_serve_cfg *cfg, int32_t n_streams, const tt_stream *streams,
                   tt_serve_stats *stats);

/* Host IQ coupling (Sec. III-A: the UEs and the gNB exchange IQ with the
 * channel through host memory over rfsim's transport).  A producer writes a
 * slot's IQ into pinned host buffer b and submits it; the library copies it
 * to HBM on its own copy stream, runs the slot (DL and UL of every listed UE,
 * one batched submission on the channel's stream) and copies the outputs back
 * to pinned host memory on a second copy stream.  `depth` buffers rotate, so
 * the copies of one slot overlap the kernels of another.  Every listed UE
 * belongs to `cell` and hears only the cell's own DL stream; taps are fed
 * through the channel as usual (their calls are ordered with the slots on
 * the channel's stream).
 * Buffer layouts, in the channel's iq_fmt, samples of one antenna contiguous:
 *   in:  the gNB's DL stream [n_ant][N], then per UE in list order [n_tx][N]
 *   out: per UE in list order its DL output [n_rx][N], then the cell's UL
 *        output [n_ant][N]. */
typedef struct {
    int32_t cell;
    int32_t n_ues;
    const int32_t *ue;                    /* [n_ues] active UE ids (copied) */
    int32_t n_samples;                    /* N per slot, <= the cell's max_samples */
    int32_t depth;                        /* slot buffers, 1 .. TT_IO_MAX_DEPTH */
} tt_io_cfg;
#define TT_IO_MAX_DEPTH 16
typedef struct tt_io tt_io;

/* Allocates depth pinned input/output buffer pairs and their HBM twins (held
 * until destroy) and two copy streams at the default priority. */
tt_status tt_io_create(tt_channel *ch, const tt_io_cfg *cfg, tt_io **out);

/* Host addresses and sizes of buffer b (owned by the io object). */
tt_status tt_io_buffers(tt_io *io, int32_t b, void **in, int64_t *in_bytes, void **out, int64_t *out_bytes);

/* Hands buffer b over: its input must be complete; the call returns at once.
 * TT_E_STATE if b is still in flight (wait for it first).  The buffer's
 * input and output must not be touched until tt_io_wait(b) returns. */
tt_status tt_io_submit(tt_io *io, int32_t b);

/* Notes the completion time of every buffer that has finished (no blocking);
 * *in_flight (optional) receives the number still in flight. */
tt_status tt_io_poll(tt_io *io, int32_t *in_flight);

/* Blocks until buffer b's outputs are in host memory.  *latency_us
 * (optional): submit to the first observation of completion (by this call,
 * tt_io_poll or tt_io_submit), or -1 if b was never submitted. */
tt_status tt_io_wait(tt_io *io, int32_t b, double *latency_us);

/* Waits for buffers in flight and frees them. NULL is a no-op. */
tt_status tt_io_destroy(tt_io *io);

/* Message for the last failure on this thread ("" if none). */
const char *tt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TT_CHANNEL_H */
