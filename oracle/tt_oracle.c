/*
 * tt_oracle.c -- plain FP64 CPU reference of the channel-emulation path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, includes or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it.  It shares no code, header, table or constant with the HIP path.
 *
 * What it computes (Tiny-Twin, Sec. III-B, the rfsim channel paragraph): each
 * receiver convolves the transmitted IQ stream with its own time-varying,
 * finite-tap channel impulse response, y_u(t) = x(t) * h_u(t), a linear
 * convolution that differs per receiver; in uplink the gNB convolves every
 * UE's stream with that UE's channel and sums the results.  Sec. IV
 * ("Tiny-Twin compatible channel traces") fixes the channel representation:
 * discrete complex taps on a fixed delay grid, one snapshot per time step,
 * and names a Jakes Doppler model for time variation.
 *
 * Discrete form written out here (the paper gives only the continuous-time
 * operator; the readings below are the ones the build takes):
 *
 *   s_r[n] = sum_{t < n_tx} sum_{l < L} h_{r,t,l}[n] * x_t[n - l]
 *
 * where n is the receiver's sample clock (n = 0 when the UE joins, x[m] = 0
 * for m < 0) and the tap is indexed by OUTPUT time n.  Tap modes, with
 * snapshot index k = floor(n / P):
 *   HOLD    h = H_k
 *   LINEAR  a = (n mod P) / P,  h = (1 - a) H_k + a H_{k+1}
 *   JAKES   h = sqrt(p_l / 16) * sum_{m<16} exp(j (2 pi frac(nu_m n) + phi_m)),
 *           nu_m = (f_D / f_s) cos((2 pi m + theta) / 16)
 * Noise: v = s + sigma * w[(off + n) mod N_pool] (w: complex FP16 pool given
 * as doubles).  ci16 output: q = clamp(round_half_even(4096 v), -32768, 32767)
 * per component.
 *
 * Sparse top-n (Sec. III-C): with nsel set, the taps of block k are those of
 * the full channel restricted to the nsel strongest taps of snapshot H_k.
 *
 * Parity status: HOLD, LINEAR, sparse selection, the FIR with its history,
 * noise and the ci16 quantiser are pinned by brute force, textbook special cases and invariants
 * (tests/test_oracle_pins.py).  JAKES is pinned statistically (mean power,
 * the J0 autocorrelation, the Doppler bound) and by its f_D = 0 special case.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

enum { TTO_HOLD = 0, TTO_LINEAR = 1, TTO_JAKES = 2 };

typedef struct {
    int32_t mode;
    int32_t L, n_tx, n_rx;
    /* HOLD / LINEAR: snapshots kbase .. kbase + nsnap - 1, layout
     * [nsnap][n_rx][n_tx][L][2] (re, im), period P samples per snapshot. */
    int64_t P;
    int64_t kbase;
    int64_t nsnap;
    const double *snaps;
    /* JAKES */
    double fd, fs;
    const double *pdp;   /* [L] */
    const double *theta; /* [n_rx][n_tx][L] */
    const double *phi;   /* [n_rx][n_tx][L][16] */
    /* Sparse top-n (HOLD / LINEAR): 0 < nsel < L keeps, per snapshot k and
     * (r, t), only the nsel taps of largest |H_k|^2 (ties: smaller l) for
     * every output of block k; 0 keeps all taps. */
    int32_t nsel;
} tto_taps;

static const double TTO_PI = 3.14159265358979323846;

static int64_t floor_div(int64_t a, int64_t b)
{
    int64_t q = a / b;
    if ((a % b != 0) && ((a < 0) != (b < 0)))
        q -= 1;
    return q;
}

static const double *snap_at(const tto_taps *tp, int64_t k, int r, int t, int l)
{
    int64_t i = k - tp->kbase;
    if (i < 0 || i >= tp->nsnap)
        return NULL;
    return tp->snaps + 2 * ((((i * tp->n_rx + r) * tp->n_tx + t) * tp->L) + l);
}

/* Whether tap l of snapshot k, pair (r, t), is among the nsel strongest
 * (Tiny-Twin, Sec. III-C, sparse convolution: only the top-n dominant taps
 * of each time step are convolved).  Strength |H|^2 = re^2 + im^2 in FP64
 * (the squares of FP32 or FP16 tap values are exact); equal strengths rank
 * the smaller delay first. */
static int tap_selected(const tto_taps *tp, int64_t k, int r, int t, int l)
{
    if (tp->nsel <= 0 || tp->nsel >= tp->L)
        return 1;
    const double *h = snap_at(tp, k, r, t, l);
    const double m = h[0] * h[0] + h[1] * h[1];
    int rank = 0;
    for (int j = 0; j < tp->L; ++j) {
        const double *g = snap_at(tp, k, r, t, j);
        const double mj = g[0] * g[0] + g[1] * g[1];
        if (mj > m || (mj == m && j < l))
            ++rank;
    }
    return rank < tp->nsel;
}

/* Channel tap h_{r,t,l}[n]; returns 0, or -1 when a needed snapshot is absent. */
int tto_tap(const tto_taps *tp, int r, int t, int l, int64_t n, double *out)
{
    if (tp->mode == TTO_HOLD || tp->mode == TTO_LINEAR) {
        int64_t k = floor_div(n, tp->P);
        const double *h0 = snap_at(tp, k, r, t, l);
        if (!h0)
            return -1;
        if (!tap_selected(tp, k, r, t, l)) {
            if (tp->mode == TTO_LINEAR && !snap_at(tp, k + 1, r, t, l))
                return -1;
            out[0] = out[1] = 0.0;
            return 0;
        }
        if (tp->mode == TTO_HOLD) {
            out[0] = h0[0];
            out[1] = h0[1];
            return 0;
        }
        const double *h1 = snap_at(tp, k + 1, r, t, l);
        if (!h1)
            return -1;
        double a = (double)(n - k * tp->P) / (double)tp->P;
        out[0] = (1.0 - a) * h0[0] + a * h1[0];
        out[1] = (1.0 - a) * h0[1] + a * h1[1];
        return 0;
    }
    if (tp->mode == TTO_JAKES) {
        double amp = sqrt(tp->pdp[l] / 16.0);
        double th = tp->theta[(r * tp->n_tx + t) * tp->L + l];
        const double *ph = tp->phi + 16 * ((r * tp->n_tx + t) * tp->L + l);
        double re = 0.0, im = 0.0;
        for (int m = 0; m < 16; ++m) {
            double nu = (tp->fd / tp->fs) * cos((2.0 * TTO_PI * m + th) / 16.0);
            double c = nu * (double)n;
            double ang = 2.0 * TTO_PI * (c - floor(c)) + ph[m];
            re += amp * cos(ang);
            im += amp * sin(ang);
        }
        out[0] = re;
        out[1] = im;
        return 0;
    }
    return -1;
}

/*
 * s_r[n0 + i] for the requested outputs.
 *   x   : [n_tx][L - 1 + N][2]; x_t[n0 - (L - 1) + j] is at j (the first L - 1
 *         entries are the stream's history, zeros before the UE joined).
 *   idx : output indices i in [0, N), or NULL for all N outputs.
 *   s   : [n_rx][n_out][2].
 * Returns 0, -1 on a missing snapshot, -2 on a bad index.
 */
int tto_fir(const tto_taps *tp, int64_t n0, int64_t N, const double *x,
            const int64_t *idx, int64_t n_out, double *s)
{
    const int L = tp->L, n_tx = tp->n_tx, n_rx = tp->n_rx;
    const int64_t xlen = (int64_t)(L - 1) + N;
    int status = 0;
    if (!idx)
        n_out = N;
#pragma omp parallel for schedule(static)
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t i = idx ? idx[o] : o;
        if (i < 0 || i >= N) {
#pragma omp atomic write
            status = -2;
            continue;
        }
        int64_t n = n0 + i;
        for (int r = 0; r < n_rx; ++r) {
            double acc_re = 0.0, acc_im = 0.0;
            for (int t = 0; t < n_tx; ++t) {
                for (int l = 0; l < L; ++l) {
                    double h[2];
                    if (tto_tap(tp, r, t, l, n, h) != 0) {
#pragma omp atomic write
                        status = -1;
                        h[0] = h[1] = 0.0;
                    }
                    const double *xv = x + 2 * (t * xlen + (L - 1) + i - l);
                    acc_re += h[0] * xv[0] - h[1] * xv[1];
                    acc_im += h[0] * xv[1] + h[1] * xv[0];
                }
            }
            s[2 * (r * n_out + o) + 0] = acc_re;
            s[2 * (r * n_out + o) + 1] = acc_im;
        }
    }
    return status;
}

/* v[o] += sigma * w[(off + n0 + i_o) mod npool] for each output o. */
void tto_add_noise(double *v, int64_t n_out, const int64_t *idx, int64_t n0,
                   double sigma, const double *pool, int64_t npool, int64_t off)
{
    for (int64_t o = 0; o < n_out; ++o) {
        int64_t i = idx ? idx[o] : o;
        int64_t p = (off + n0 + i) % npool;
        if (p < 0)
            p += npool;
        v[2 * o + 0] += sigma * pool[2 * p + 0];
        v[2 * o + 1] += sigma * pool[2 * p + 1];
    }
}

/* ci16 output: q = clamp(rne(4096 v)) per component; returns saturated count. */
int64_t tto_quantize_ci16(const double *v, int64_t n_values, int16_t *q)
{
    int64_t sat = 0;
    for (int64_t i = 0; i < n_values; ++i) {
        double y = nearbyint(4096.0 * v[i]); /* default rounding: to nearest, ties to even */
        if (y > 32767.0) {
            y = 32767.0;
            ++sat;
        } else if (y < -32768.0) {
            y = -32768.0;
            ++sat;
        }
        q[i] = (int16_t)y;
    }
    return sat;
}

void tto_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int tto_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
