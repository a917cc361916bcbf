/*
 * oracle.c -- plain FP64 CPU oracle for the readout channelizer (polyphase
 * filter bank) and the direct-demodulation (DDC) bank of
 * Minutolo et al., "A flexible GPU-accelerated radio-frequency readout for
 * superconducting detectors" (arXiv:1812.02200).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file's library: it is used by tests/, by the smoke check and by
 * the CPU-baseline leg of the benchmark.  It shares no code, header, table or
 * constant with the HIP implementation.
 *
 * Everything is computed from the plain definitions, in double precision,
 * one output at a time, with sums taken in ascending index order.  OpenMP
 * parallelises over independent outputs only, so results do not depend on
 * the thread count.
 *
 * Notation (x[m] = I[m] + j Q[m], I at even int16 index, Q at odd):
 *
 * PFB (paper Sec. III.A): a prototype FIR h of length N*M (N channels = the
 * decimation factor, M taps per channel; the paper's A_v).  Frame p exists
 * when p*N + N*M <= S ("valid" frames only) and is
 *     v_p[n] = sum_{m=0}^{M-1} h[m*N + n] * x[p*N + m*N + n],   n in [0,N)
 *     X_p[k] = sum_{n=0}^{N-1} v_p[n] * exp(-2 pi i k n / N),   k in [0,N)
 * i.e. the section of N*M samples is weighted by the FIR, folded to N points
 * and Fourier transformed (bins in natural order, no 1/N, no fftshift).
 *
 * DDC (paper Sec. III.B): per tone t a numerically controlled oscillator with
 * a 64-bit phase phi_t[m] = phi0_t + m*inc_t (mod 2^64, m the absolute sample
 * index), a 2^16-entry cos/sin table addressed by idx = phi >> 48
 * (truncation), a mix z_t[m] = x[m] * conj(c_t[m]), a T-tap low-pass and
 * decimation by D:
 *     y_t[n] = sum_{k=0}^{T-1} h[k] * z_t[n*D + T-1-k],  for n*D + T-1 <= S-1.
 * The paper's own anti-alias filter (a moving average) is the special case
 * h = 1/D, T = D.
 *
 * Chirped tones (paper Sec. III.C, Eq. 1: phase 2 pi (f0 t + k t^2)): the
 * phase becomes quadratic in the sample index,
 *     phi_t[m] = phi0_t + m*inc_t + K_t * m(m-1)/2   (mod 2^64),
 * the closed form of a second-order accumulator (phase += rate; rate += K).
 * Sampling Eq. 1 at t = m/fs gives exactly this with inc = (f0/fs + k/fs^2)
 * 2^64 and K = (2k/fs^2) 2^64: Eq. 1 is taken as printed, so the
 * instantaneous frequency f0 + 2kt ramps at 2k.  K = 0 is the linear NCO.
 *
 * Tx (the DAC buffers the GPU generates, Sec. III; chirps, Sec. III.C): the
 * sum over tones of amplitude times the same table value, rounded to int16
 * DAC words -- see orc_tx below.
 *
 * Parity status: every function here is pinned by the CPU tests in
 * tests/test_oracle_pins.py (closed forms, brute force, library routines,
 * invariants); none is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TWO_PI 6.283185307179586476925286766559

/* ---------------------------------------------------------------- helpers */

/* Sample m of the stream: from interleaved int16 I/Q, or from a complex
 * double array (re, im interleaved) when iq is NULL. */
static inline void orc_sample(const int16_t *iq, const double *xc, int64_t m,
                              double *re, double *im)
{
    if (iq) {
        *re = (double)iq[2 * m];
        *im = (double)iq[2 * m + 1];
    } else {
        *re = xc[2 * m];
        *im = xc[2 * m + 1];
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------ DFT */

/* Direct DFT by its definition, O(N^2):
 *     X[k] = sum_n x[n] exp(-2 pi i k n / N).
 * The exponent k*n is reduced mod N in integers before forming the angle, so
 * every twiddle is cos/sin of an angle in [0, 2 pi).  x, X: N complex values,
 * (re, im) interleaved; x and X must not overlap. */
void orc_dft_direct(const double *x, int64_t N, double *X)
{
    for (int64_t k = 0; k < N; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t n = 0; n < N; ++n) {
            int64_t e = (k * n) % N;
            double a = -ORC_TWO_PI * (double)e / (double)N;
            double c = cos(a), s = sin(a);
            double xr = x[2 * n], xi = x[2 * n + 1];
            sr += xr * c - xi * s;
            si += xr * s + xi * c;
        }
        X[2 * k] = sr;
        X[2 * k + 1] = si;
    }
}

/* Textbook iterative radix-2 FFT (bit-reversal permutation, then butterfly
 * stages of length 2, 4, ..., N), in place, same sign and scaling as
 * orc_dft_direct.  Every twiddle exp(-2 pi i j / len) is evaluated directly
 * with cos/sin (no recurrence).  N must be a power of two. */
void orc_fft_pow2(double *x, int64_t N)
{
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < N; ++i) {
        int64_t bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double tr = x[2 * i], ti = x[2 * i + 1];
            x[2 * i] = x[2 * j];
            x[2 * i + 1] = x[2 * j + 1];
            x[2 * j] = tr;
            x[2 * j + 1] = ti;
        }
    }
    for (int64_t len = 2; len <= N; len <<= 1) {
        int64_t half = len >> 1;
        for (int64_t j = 0; j < half; ++j) {
            double a = -ORC_TWO_PI * (double)j / (double)len;
            double wr = cos(a), wi = sin(a);
            for (int64_t b = 0; b < N; b += len) {
                double *u = x + 2 * (b + j);
                double *v = x + 2 * (b + j + half);
                double tr = v[0] * wr - v[1] * wi;
                double ti = v[0] * wi + v[1] * wr;
                v[0] = u[0] - tr;
                v[1] = u[1] - ti;
                u[0] += tr;
                u[1] += ti;
            }
        }
    }
}

static int orc_is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* DFT of one frame in place: the radix-2 FFT for powers of two, the direct
 * definition otherwise.  tmp: 2*N doubles of scratch. */
static void orc_dft_frame(double *v, int64_t N, double *tmp)
{
    if (orc_is_pow2(N)) {
        orc_fft_pow2(v, N);
    } else {
        orc_dft_direct(v, N, tmp);
        memcpy(v, tmp, sizeof(double) * 2 * (size_t)N);
    }
}

/* ------------------------------------------------------------------ PFB */

/* Number of valid frames in S samples: frame p needs samples [pN, pN+NM). */
int64_t orc_pfb_nframes(int64_t S, int64_t N, int64_t M)
{
    if (N <= 0 || M <= 0 || S < N * M) return 0;
    return (S - N * M) / N + 1;
}

/* Fold step of frame p (paper Sec. III.A: weight an N*M-sample section by
 * the FIR and sum the M sub-sections of length N):
 *     v[n] = sum_{m=0}^{M-1} h[m*N + n] * x[p*N + m*N + n]. */
static void orc_pfb_fold(const int16_t *iq, const double *xc, int64_t p,
                         int64_t N, int64_t M, const double *h, double *v)
{
    for (int64_t n = 0; n < N; ++n) {
        double sr = 0.0, si = 0.0;
        for (int64_t m = 0; m < M; ++m) {
            double xr, xi;
            orc_sample(iq, xc, p * N + m * N + n, &xr, &xi);
            double w = h[m * N + n];
            sr += w * xr;
            si += w * xi;
        }
        v[2 * n] = sr;
        v[2 * n + 1] = si;
    }
}

/* PFB output for a list of frames (frames == NULL: frames 0..nf-1).
 * Input: iq (interleaved int16, S samples) or, when iq is NULL, xc (complex
 * double).  h: N*M prototype taps.  out: nf*N complex values, frame-major.
 * Frames that do not exist in S samples are written as NaN. */
void orc_pfb_frames(const int16_t *iq, const double *xc, int64_t S, int64_t N,
                    int64_t M, const double *h, const int64_t *frames,
                    int64_t nf, double *out)
{
    int64_t total = orc_pfb_nframes(S, N, M);
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * 2 * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < nf; ++i) {
            int64_t p = frames ? frames[i] : i;
            double *v = out + 2 * N * i;
            if (p < 0 || p >= total) {
                for (int64_t k = 0; k < 2 * N; ++k) v[k] = NAN;
                continue;
            }
            orc_pfb_fold(iq, xc, p, N, M, h, v);
            orc_dft_frame(v, N, tmp);
        }
        free(tmp);
    }
}

/* Only the fold (FIR) step, for the precision report and for pins that
 * check the DFT stage against a library FFT. */
void orc_pfb_fold_frames(const int16_t *iq, const double *xc, int64_t S,
                         int64_t N, int64_t M, const double *h,
                         const int64_t *frames, int64_t nf, double *out)
{
    int64_t total = orc_pfb_nframes(S, N, M);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nf; ++i) {
        int64_t p = frames ? frames[i] : i;
        double *v = out + 2 * N * i;
        if (p < 0 || p >= total) {
            for (int64_t k = 0; k < 2 * N; ++k) v[k] = NAN;
            continue;
        }
        orc_pfb_fold(iq, xc, p, N, M, h, v);
    }
}

/* Selected channels only (the paper's option of returning chosen channels
 * instead of the whole spectrum, Sec. III.A): the same fold, then
 * X_p[k] = sum_n v_p[n] exp(-2 pi i k n / N) summed directly for each
 * requested k (an evaluation independent of the FFT above).
 * out[(i*nsel + c)*2 + {0,1}] for frame i and channel chans[c]. */
void orc_pfb_channels(const int16_t *iq, const double *xc, int64_t S, int64_t N,
                      int64_t M, const double *h, const int64_t *chans,
                      int64_t nsel, double *out)
{
    int64_t nf = orc_pfb_nframes(S, N, M);
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * 2 * (size_t)N);
#pragma omp for schedule(static)
        for (int64_t p = 0; p < nf; ++p) {
            orc_pfb_fold(iq, xc, p, N, M, h, v);
            for (int64_t c = 0; c < nsel; ++c) {
                int64_t k = chans[c];
                double sr = 0.0, si = 0.0;
                for (int64_t n = 0; n < N; ++n) {
                    /* angle reduced exactly: k*n mod N */
                    double a = -ORC_TWO_PI * (double)((k * n) % N) / (double)N;
                    double cr = cos(a), ci = sin(a);
                    sr += v[2 * n] * cr - v[2 * n + 1] * ci;
                    si += v[2 * n] * ci + v[2 * n + 1] * cr;
                }
                out[2 * (p * nsel + c)] = sr;
                out[2 * (p * nsel + c) + 1] = si;
            }
        }
        free(v);
    }
}

/* ------------------------------------------------------------------ DDC */

/* The NCO's cos/sin table in FP64 at the quantised angles:
 * tab[2i] = cos(2 pi i / 2^16), tab[2i+1] = sin(2 pi i / 2^16). */
void orc_nco_table(double *tab)
{
    for (int64_t i = 0; i < 65536; ++i) {
        double a = ORC_TWO_PI * (double)i / 65536.0;
        tab[2 * i] = cos(a);
        tab[2 * i + 1] = sin(a);
    }
}

/* Phase of the NCO at absolute sample m: phi0 + m*inc in 64-bit wrap-around
 * arithmetic (unsigned overflow is the mod 2^64 reduction). */
uint64_t orc_nco_phase(uint64_t phi0, uint64_t inc, uint64_t m)
{
    return phi0 + m * inc;
}

/* m(m-1)/2 mod 2^64, exactly: halve whichever factor is even first. */
static uint64_t orc_tri(uint64_t m)
{
    if (m == 0) return 0;
    return (m % 2 == 0) ? (m / 2) * (m - 1) : m * ((m - 1) / 2);
}

/* Phase of a chirped NCO at absolute sample m (K = 0: linear). */
uint64_t orc_chirp_phase(uint64_t phi0, uint64_t inc, uint64_t K, uint64_t m)
{
    return phi0 + m * inc + K * orc_tri(m);
}

/* Phases after S samples, one per tone. */
void orc_nco_phases(const uint64_t *phi0, const uint64_t *inc, int64_t ntones,
                    uint64_t S, uint64_t *out)
{
    for (int64_t t = 0; t < ntones; ++t)
        out[t] = orc_nco_phase(phi0 ? phi0[t] : 0, inc[t], S);
}

/* Number of outputs in S samples: output n covers samples [nD, nD+T-1]. */
int64_t orc_ddc_noutputs(int64_t S, int64_t T, int64_t D)
{
    if (T <= 0 || D <= 0 || S < T) return 0;
    return (S - T) / D + 1;
}

/* One output y_t[n].  exact_nco = 0: c = table value at idx = phi >> 48
 * (the method); exact_nco = 1: c = exp(i 2 pi phi / 2^64) without
 * truncation (used only to bound the truncation error in tests). */
static void orc_ddc_one(const int16_t *iq, const double *xc, uint64_t inc,
                        uint64_t phi0, uint64_t K, int64_t T, const double *h,
                        int64_t D, int64_t n, int exact_nco, const double *tab,
                        double *yr, double *yi)
{
    double sr = 0.0, si = 0.0;
    for (int64_t k = 0; k < T; ++k) {
        int64_t m = n * D + T - 1 - k;
        uint64_t phi = orc_chirp_phase(phi0, inc, K, (uint64_t)m);
        double cr, ci;
        if (exact_nco) {
            double a = ORC_TWO_PI * ((double)phi / 18446744073709551616.0);
            cr = cos(a);
            ci = sin(a);
        } else {
            uint64_t idx = phi >> 48;
            cr = tab[2 * idx];
            ci = tab[2 * idx + 1];
        }
        double xr, xi;
        orc_sample(iq, xc, m, &xr, &xi);
        /* z = x * conj(c) */
        double zr = xr * cr + xi * ci;
        double zi = xi * cr - xr * ci;
        sr += h[k] * zr;
        si += h[k] * zi;
    }
    *yr = sr;
    *yi = si;
}

/* All outputs of all tones: out[(t*nout + n)*2 + {0,1}], tone-major.
 * phi0 and chirp (K per tone) may be NULL (all zero).  Returns nout. */
int64_t orc_ddc(const int16_t *iq, const double *xc, int64_t S, int64_t ntones,
                const uint64_t *inc, const uint64_t *phi0, const uint64_t *chirp,
                int64_t T, const double *h, int64_t D, int exact_nco, double *out)
{
    int64_t nout = orc_ddc_noutputs(S, T, D);
    double *tab = (double *)malloc(sizeof(double) * 2 * 65536);
    orc_nco_table(tab);
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t t = 0; t < ntones; ++t)
        for (int64_t n = 0; n < nout; ++n) {
            double *y = out + 2 * (t * nout + n);
            orc_ddc_one(iq, xc, inc[t], phi0 ? phi0[t] : 0, chirp ? chirp[t] : 0,
                        T, h, D, n, exact_nco, tab, &y[0], &y[1]);
        }
    free(tab);
    return nout;
}

/* Selected outputs (tone_idx[i], out_idx[i]) for sampled checks of large
 * runs; points outside the valid range are written as NaN. */
void orc_ddc_points(const int16_t *iq, const double *xc, int64_t S,
                    const uint64_t *inc, const uint64_t *phi0,
                    const uint64_t *chirp, int64_t T,
                    const double *h, int64_t D, const int64_t *tone_idx,
                    const int64_t *out_idx, int64_t npts, int exact_nco,
                    double *out)
{
    int64_t nout = orc_ddc_noutputs(S, T, D);
    double *tab = (double *)malloc(sizeof(double) * 2 * 65536);
    orc_nco_table(tab);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        int64_t t = tone_idx[i], n = out_idx[i];
        if (n < 0 || n >= nout) {
            out[2 * i] = NAN;
            out[2 * i + 1] = NAN;
            continue;
        }
        orc_ddc_one(iq, xc, inc[t], phi0 ? phi0[t] : 0, chirp ? chirp[t] : 0,
                    T, h, D, n, exact_nco, tab, &out[2 * i], &out[2 * i + 1]);
    }
    free(tab);
}

/* ------------------------------------------------------------------- Tx */

/* Multi-tone transmit synthesis, the DDC's inverse (the GPU produces the
 * DAC buffers, paper Sec. III; chirped excitations, Sec. III.C): tone t
 * carries an oscillator state at the buffer's first sample -- phase phi_t,
 * rate r_t (phase step to the next sample) and second difference K_t -- and
 * a real amplitude a_t in DAC counts.  Sample j of the buffer is
 *     v[j] = sum_t a_t * Tab32[(phi_t + j r_t + K_t j(j-1)/2) >> 48]
 * with Tab32 the FP32 cos/sin table of the DDC (defined through the quarter
 * wave q[j] = fp32(sin(pi j / 2^15))), and the DAC word is v rounded to the
 * nearest integer (ties to even) and saturated to int16, I and Q
 * interleaved.  Because a rounding of floating-point values decides an
 * integer here, the sum is formed in the FP32 precision of the device, in
 * ascending tone order, each term a single-rounded FP32 product and each
 * addition a single-rounded FP32 sum starting from +0.  After the buffer the
 * state advances by n samples: phi += n r + K n(n-1)/2, r += n K. */

/* The FP32 table by its definition: quadrant g = i >> 14, r = i mod 2^14. */
void orc_tab32(float *tab)
{
    float q[(1 << 14) + 1];
    for (int j = 0; j <= (1 << 14); ++j) q[j] = (float)sin(3.14159265358979323846 * (double)j / 32768.0);
    for (int i = 0; i < 65536; ++i) {
        int g = i >> 14, r = i & 0x3fff;
        float c = q[(1 << 14) - r], s = q[r];
        float co, si;
        switch (g) {
        case 0: co = c;  si = s;  break;
        case 1: co = -s; si = c;  break;
        case 2: co = -c; si = -s; break;
        default: co = s; si = -c; break;
        }
        tab[2 * i] = co;
        tab[2 * i + 1] = si;
    }
}

static int16_t orc_dac(float v)
{
    float r = rintf(v);               /* ties to even (default rounding mode) */
    if (r > 32767.0f) return 32767;
    if (r < -32768.0f) return -32768;
    return (int16_t)r;
}

void orc_tx(int64_t ntones, const uint64_t *phase, const uint64_t *rate,
            const uint64_t *chirp, const float *amp, int64_t n, int16_t *out)
{
    float *tab = (float *)malloc(sizeof(float) * 2 * 65536);
    orc_tab32(tab);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        float vr = 0.0f, vi = 0.0f;
        for (int64_t t = 0; t < ntones; ++t) {
            uint64_t ph = phase[t] + (uint64_t)j * rate[t] + (chirp ? chirp[t] * orc_tri((uint64_t)j) : 0);
            uint64_t idx = ph >> 48;
            float pr = amp[t] * tab[2 * idx];
            float pi = amp[t] * tab[2 * idx + 1];
            vr = vr + pr;
            vi = vi + pi;
        }
        out[2 * j] = orc_dac(vr);
        out[2 * j + 1] = orc_dac(vi);
    }
    free(tab);
}

/* Oscillator state after n samples. */
void orc_tx_advance(int64_t ntones, uint64_t *phase, uint64_t *rate,
                    const uint64_t *chirp, uint64_t n)
{
    for (int64_t t = 0; t < ntones; ++t) {
        uint64_t K = chirp ? chirp[t] : 0;
        phase[t] = phase[t] + n * rate[t] + K * orc_tri(n);
        rate[t] = rate[t] + n * K;
    }
}
