/*
 * rfchan.h -- C ABI of the MI355X (gfx950) readout channelizer and demodulator.
 *
 * Implements the GPU signal-processing hot path of Minutolo et al., "A flexible
 * GPU-accelerated radio-frequency readout for superconducting detectors"
 * (arXiv:1812.02200): a critically sampled polyphase filter bank (Sec. III.A)
 * and a bank of direct demodulators (Sec. III.B), on a continuous stream of
 * complex-baseband int16 I/Q samples (the 14-bit, 200 Ms/s ADC stream of
 * Sec. II.A).  Filter history and oscillator phase stay on the device between
 * calls, so a stream may be cut into buffers of any size.
 *
 * Conventions shared by every call:
 *  - Samples are interleaved int16 I/Q in device memory: I[m] at index 2m,
 *    Q[m] at 2m+1, x[m] = I[m] + j Q[m].  Pointers must be 4-byte aligned
 *    (16-byte alignment gives the fastest loads).
 *  - Outputs are complex64: float pairs (re, im), interleaved.
 *  - Work is asynchronous on the HIP stream passed as `hip_stream`
 *    (a hipStream_t; NULL means the default stream).  Successive calls on one
 *    handle are ordered even if they name different streams.  The caller owns
 *    every buffer it passes and keeps it alive until the stream has reached
 *    the work.
 *  - Every call returns a status (RF_OK = 0).  A call that fails leaves the
 *    handle's state unchanged.  Nothing throws across the ABI.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Device memory is allocated only by the *_create calls; *_process calls
 *    never allocate.
 */
#ifndef RFCHAN_H
#define RFCHAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define RF_OK 0
#define RF_EINVAL 1        /* invalid argument (null pointer, bad size, ...) */
#define RF_ENOMEM 2        /* device or host allocation failed */
#define RF_EDEVICE 3       /* a HIP runtime call failed (see rf_last_error) */
#define RF_ECAPACITY 4     /* output buffer too small for this call */
#define RF_EAGAIN 5        /* resource busy / does not fit now; retry later */
#define RF_EUNSUPPORTED 6  /* valid request this build does not support */

/* Short description of a status code (static string). */
const char *rf_strerror(int status);

/* Detail of the most recent failure on the calling thread ("" if none). */
const char *rf_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int rf_version(void);

/* ============================================================ PFB channelizer
 *
 * Critically sampled polyphase filter bank (paper Sec. III.A): N channels,
 * decimation N, a prototype FIR of length N*M (M taps per channel).  Frame p
 * of the stream covers samples [p*N, p*N + N*M) and is
 *     v_p[n] = sum_{m=0}^{M-1} h[m*N + n] * x[p*N + m*N + n],   n in [0, N)
 *     X_p[k] = sum_{n=0}^{N-1} v_p[n] * exp(-2 pi i k n / N),   k in [0, N)
 * (unnormalised forward DFT, bins in natural order: bin k >= N/2 is the
 * negative frequency (k - N) fs / N).  Only frames whose N*M samples have all
 * arrived are emitted, so the first frame appears once N*M samples exist.
 */
typedef struct rf_pfb *rf_pfb_t;

/* DFT stage implementations. */
#define RF_DFT_FFT_F32 0      /* FP32 FFT (radix-4/16 Stockham in LDS)                  */
#define RF_DFT_MFMA_F16X2 1   /* DFT as GEMMs on FP16 MFMA, hi/lo split operands, N=16..256 */
#define RF_DFT_MFMA_BF16X2 2  /* DFT as GEMMs on BF16 MFMA, hi/lo split operands, N=16..256 */

/* Create a channelizer on the current HIP device.
 *   out       receives the handle.
 *   nchan     N: a power of two, 16 <= N <= 4096 (one fused kernel per buffer),
 *             or any N in [16, 2^24] whose only prime factors are 2, 3 and 5 and
 *             that splits into two factors <= 4096 -- e.g. the 10^5 channels of
 *             Sec. III.A, Fig. 3 -- (a fold pass and a four-step FFT through
 *             device scratch of 2 x (max_samples_per_call/N + 2) frames; FP32 FFT
 *             mode only; no chosen channels, no tuning, not served).
 *   ntaps     M: 1 <= M <= 16.
 *   proto     host array of N*M FP32 prototype taps h[0..N*M); copied, the
 *             caller may free it on return.
 *   dft_mode  one of RF_DFT_*; the MFMA modes need N in {16, 32, 64, 128,
 *             256} (RF_EUNSUPPORTED otherwise).  They factor N = 16 N2 into a
 *             DFT16 product and a block-diagonal DFT_N2 product, each on MFMA
 *             with both operands split into high and low half-precision parts
 *             (hi*hi + hi*lo + lo*hi, FP32 accumulation).  The taps are
 *             stored multiplied by an exact power of two, chosen from the
 *             largest column sum of |h| so that no half-precision operand can
 *             exceed 2^15 for any int16 input, and the outputs are scaled
 *             back exactly: any finite prototype is accepted (RF_EUNSUPPORTED
 *             only if that power of two would leave [2^-100, 2^100]).
 *   max_samples_per_call  largest nsamples a single pfb_process will accept
 *             (>= 1).  Bounds the work of one call; no memory scales with it.
 * Allocates all device state (taps, twiddles, two history buffers of N*M
 * samples).  Returns RF_EINVAL for bad sizes, RF_ENOMEM / RF_EDEVICE on
 * allocation or copy failure. */
int pfb_create(rf_pfb_t *out, int32_t nchan, int32_t ntaps, const float *proto,
               int32_t dft_mode, uint64_t max_samples_per_call);

/* Number of frames the next pfb_process of `nsamples` samples will emit; a
 * pure host-side function of the handle's sample count (no device sync). */
uint64_t pfb_frames_for(rf_pfb_t pfb, uint64_t nsamples);

/* Choose the channels pfb_process returns (paper Sec. III.A: the full
 * spectrum or specific user-defined channels).  channels: host [nsel]
 * distinct bins in [0, N) in the order wanted; after this call every frame
 * is written as nsel complex values, frame f's value for channels[c] at
 * out_dev[f*nsel + c] -- bit-identical to the same bin of the full spectrum
 * (the transform is the same; only the chosen bins are stored).  nsel = 0
 * (channels may be NULL) returns to all N bins in natural order.  Frame
 * counts, history and state are unaffected.  RF_EINVAL for a bin out of
 * range or repeated; RF_EUNSUPPORTED for the MFMA DFT modes.  Waits for the
 * handle's last stream. */
int pfb_set_channels(rf_pfb_t pfb, const int32_t *channels, int32_t nsel);

/* Channelize the next `nsamples` samples of the stream.
 *   iq_dev          device pointer, 2*nsamples int16 (may be NULL if nsamples == 0).
 *   nsamples        any value from 0 to max_samples_per_call, including < N.
 *   out_dev         device pointer to out_cap_frames * N complex64 values; frame
 *                   f of this call is written at out_dev + 2*N*f (frame-major;
 *                   N becomes nsel after pfb_set_channels).
 *   out_cap_frames  capacity in frames (of N values, or of nsel values after
 *                   pfb_set_channels); RF_ECAPACITY if < pfb_frames_for().
 *   frames_out      host pointer (may be NULL): number of frames written.
 *   hip_stream      hipStream_t to enqueue on.
 * Enqueues one kernel; returns without waiting for it. */
int pfb_process(rf_pfb_t pfb, const int16_t *iq_dev, uint64_t nsamples, float *out_dev,
                uint64_t out_cap_frames, uint64_t *frames_out, void *hip_stream);

/* pfb_process for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Arguments, results, ordering and errors are those of pfb_process, and the
 * output is bit-identical to it; the only difference is where a large or
 * non-power-of-two-N handle's kernels keep their scratch (the folded frames
 * and the first FFT step's output): in a 64 MiB array that the library holds
 * in each GPU's memory from its first use on that GPU until the process ends,
 * shared by every such call on that GPU, instead of in the handle.  The call
 * allocates nothing.  Power-of-two-N handles use no scratch and are processed
 * exactly as by pfb_process.
 *   RF_EINVAL when the call's frames need more than the 64 MiB: F * N * 8
 *   bytes for one-step N, twice that (each part rounded up to 256 bytes) for
 *   two-step N, with F = pfb_frames_for(nsamples); the handle is unchanged.
 * Calls on one GPU that can overlap in time -- on different HIP streams,
 * or from different threads -- race on the shared array; order them on one
 * stream. */
int pfb_process_static(rf_pfb_t pfb, const int16_t *iq_dev, uint64_t nsamples, float *out_dev,
                       uint64_t out_cap_frames, uint64_t *frames_out, void *hip_stream);

/* Counters of the stream so far (host-side, no sync). Any pointer may be NULL. */
int pfb_counters(rf_pfb_t pfb, uint64_t *samples_in, uint64_t *frames_out,
                 uint64_t *history_samples);

/* Exact checkpoint of the stream state (history samples and counters).
 * pfb_get_state: if blob is NULL or *size is too small, sets *size to the
 * required size and returns RF_ECAPACITY (RF_OK when blob is NULL);
 * otherwise waits for the handle's last stream and copies the state out.
 * pfb_set_state: restores a blob from a handle with the same N and M
 * (RF_EINVAL otherwise); waits for the handle's last stream first. */
int pfb_get_state(rf_pfb_t pfb, void *blob, size_t *size);
int pfb_set_state(rf_pfb_t pfb, const void *blob, size_t size);

/* Forget the stream: empty history, counters to zero (waits for pending work). */
int pfb_reset(rf_pfb_t pfb);

/* Wait for pending work and free the handle (NULL is accepted). */
int pfb_destroy(rf_pfb_t pfb);

/* ============================================================ DDC bank
 *
 * Direct demodulation of a set of tones (paper Sec. III.B).  Tone t has a
 * 64-bit integer phase accumulator: at absolute sample m its phase is
 *     phi_t[m] = phase0[t] + m * phase_inc[t]   (mod 2^64),
 * the oscillator value is c_t[m] = Tab[phi_t[m] >> 48] from a 2^16-entry FP32
 * cos/sin table (truncation, no interpolation), and the output is
 *     y_t[n] = sum_{k=0}^{T-1} h[k] * x[n*D + T-1-k] * conj(c_t[n*D + T-1-k])
 * for every n with n*D + T - 1 < samples received: mix down, a T-tap FIR
 * low-pass (the paper's moving average is h = 1/D, T = D) and decimation by D.
 * Tab[i] = (cos, sin)(2 pi i / 2^16) rounded to FP32, defined through the
 * quarter wave q[j] = fp32(sin(pi j / 2^15)), j = 0..2^14, by symmetry.
 * A tone at frequency f of a stream sampled at fs has
 * phase_inc = round(f / fs * 2^64) mod 2^64.
 */
typedef struct rf_ddc *rf_ddc_t;

/* Create a demodulator bank on the current HIP device.
 *   ntones     1 <= ntones <= 65536.
 *   phase_inc  host array [ntones] of 64-bit tuning words (copied).
 *   phase0     host array [ntones] of initial phases, or NULL for all zero.
 *   ntaps      T: 1 <= T <= 4096.
 *   lpf        host array [T] of FP32 low-pass taps h[0..T) (copied).
 *   decim      D: 1 <= D <= 2^20.
 *   max_samples_per_call  largest nsamples one ddc_process accepts (>= 1).
 * Returns RF_EINVAL / RF_ENOMEM / RF_EDEVICE as pfb_create. */
int ddc_create(rf_ddc_t *out, int32_t ntones, const uint64_t *phase_inc,
               const uint64_t *phase0, int32_t ntaps, const float *lpf, int32_t decim,
               uint64_t max_samples_per_call);

/* Create a bank of chirped tones (paper Sec. III.C, Eq. 1: a tone whose phase
 * is quadratic in time, 2 pi (f0 t + k t^2)).  Tone t's phase at absolute
 * sample m is
 *     phi_t[m] = phase0[t] + m * phase_inc[t] + chirp[t] * m(m-1)/2  (mod 2^64),
 * i.e. a second-order accumulator: the phase advances by a rate that itself
 * advances by chirp[t] each sample.  Eq. 1 sampled at t = m/fs is exactly this
 * with phase_inc = (f0/fs + k/fs^2) 2^64 and chirp = (2k/fs^2) 2^64, each
 * rounded mod 2^64 (Eq. 1 taken as printed: the instantaneous frequency
 * f0 + 2kt ramps at 2k).  chirp[t] = 0 is an ordinary tone.  Everything else
 * -- table, mix, low-pass, decimation, ddc_process, state, phase read-back
 * (ddc_get_phase returns phi_t at the next sample) -- is as for ddc_create.
 *   chirp      host array [ntones] of 64-bit second-difference words (copied);
 *              NULL makes this call identical to ddc_create.
 * Other arguments and errors as ddc_create.  Chirped banks are not accepted
 * by the serving API (rfs_*), whose stream descriptor has no chirp words. */
int ddc_create_chirp(rf_ddc_t *out, int32_t ntones, const uint64_t *phase_inc,
                     const uint64_t *phase0, const uint64_t *chirp, int32_t ntaps,
                     const float *lpf, int32_t decim, uint64_t max_samples_per_call);

/* Outputs per tone that the next ddc_process of `nsamples` samples emits. */
uint64_t ddc_outputs_for(rf_ddc_t ddc, uint64_t nsamples);

/* Demodulate the next `nsamples` samples.
 *   out_dev  device pointer; output n of tone t (n counted from this call's
 *            first output) is written at out_dev + 2*(t*ld + n): tone-major.
 *   ld       row stride in complex values, >= ddc_outputs_for(nsamples)
 *            (RF_ECAPACITY otherwise).
 *   nout     host pointer (may be NULL): outputs per tone written.
 * Enqueues one kernel on hip_stream and returns. */
int ddc_process(rf_ddc_t ddc, const int16_t *iq_dev, uint64_t nsamples, float *out_dev,
                uint64_t ld, uint64_t *nout, void *hip_stream);

/* Phase of every tone at the next unreceived sample, phase0 + S*phase_inc
 * (mod 2^64), as computed on the device by the last ddc_process; waits for the
 * handle's last stream.  phase_host: host array [ntones]. */
int ddc_get_phase(rf_ddc_t ddc, uint64_t *phase_host);

/* Counters (host-side, no sync). Any pointer may be NULL. */
int ddc_counters(rf_ddc_t ddc, uint64_t *samples_in, uint64_t *outputs_out,
                 uint64_t *history_samples);

/* Checkpoint / restore / reset / free, with the semantics of the pfb_ calls.
 * A state blob restores onto a bank with the same ntones, tuning words,
 * phases, taps and decimation. */
int ddc_get_state(rf_ddc_t ddc, void *blob, size_t *size);
int ddc_set_state(rf_ddc_t ddc, const void *blob, size_t size);
int ddc_reset(rf_ddc_t ddc);
int ddc_destroy(rf_ddc_t ddc);

/* ============================================================ Tx synthesis
 *
 * The transmit buffers (DAC words) the readout generates on the GPU (paper
 * Sec. III: the transmission-buffer producer; Sec. III.C: chirped
 * excitations, Eq. 1), the DDC's inverse.  Tone t carries an oscillator
 * state -- phase phi_t, rate r_t (phase step to the next sample) and second
 * difference K_t (0 for a fixed tone) -- and an amplitude a_t in DAC counts.
 * With the state at a buffer's first sample, its sample j is
 *     v[j] = sum_t a_t * Tab[(phi_t + j r_t + K_t j(j-1)/2) >> 48]
 * (Tab as for the DDC bank), formed in FP32 in ascending tone order with
 * every product and every partial sum rounded to FP32 (no fused
 * multiply-add), then rounded to the nearest integer (ties to even) and
 * saturated to [-32768, 32767]; I and Q are interleaved int16 as on the
 * receive side.  After a buffer of n samples the state advances to
 * phi += n r + K n(n-1)/2, r += n K, so consecutive buffers form one
 * continuous waveform.  A fixed tone of frequency f has r = round(f/fs 2^64);
 * an Eq. 1 chirp has the words of ddc_create_chirp.
 */
typedef struct rf_tx *rf_tx_t;

/* Create a transmit bank on the current HIP device.
 *   ntones     1 <= ntones <= 65536.
 *   phase_inc  host [ntones]: initial rates r_t (copied).
 *   phase0     host [ntones]: initial phases, or NULL for all zero.
 *   chirp      host [ntones]: second differences K_t, or NULL (fixed tones;
 *              the bank then cannot take chirp words later).
 *   amplitude  host [ntones]: a_t in DAC counts, finite (copied).
 *   max_samples_per_call  largest nsamples one tx_synthesize accepts.
 * Returns RF_EINVAL for bad arguments, RF_ENOMEM / RF_EDEVICE on failure. */
int tx_create(rf_tx_t *out, int32_t ntones, const uint64_t *phase_inc, const uint64_t *phase0,
              const uint64_t *chirp, const float *amplitude, uint64_t max_samples_per_call);

/* Write the next nsamples of the waveform to out_dev (device, 2*nsamples
 * int16, 4-byte aligned, owned by the caller and kept live until the stream
 * reaches the work) and advance the state.  Asynchronous on hip_stream,
 * ordered after the handle's previous call.  nsamples = 0 does nothing;
 * nsamples > max_samples_per_call is RF_EINVAL. */
int tx_synthesize(rf_tx_t tx, int16_t *out_dev, uint64_t nsamples, void *hip_stream);

/* Feedback (paper Sec. III: the buffer generator changes its output in
 * response to the processed signal): replace the amplitudes, the current
 * rates and/or the second differences (each array host [ntones], NULL keeps
 * the current values) from the next sample on; the phase continues without
 * a jump.  Waits for the handle's last stream.  chirp on a bank created
 * without chirp words is RF_EINVAL; non-finite amplitudes are RF_EINVAL. */
int tx_set_tones(rf_tx_t tx, const float *amplitude, const uint64_t *phase_inc, const uint64_t *chirp);

/* Oscillator state at the next sample (host arrays [ntones], each may be
 * NULL) and the number of samples produced.  Waits for the last stream. */
int tx_get_state(rf_tx_t tx, uint64_t *phase, uint64_t *rate, uint64_t *samples);

/* Back to the creation state (phases, rates, second differences,
 * amplitudes, sample count 0). */
int tx_reset(rf_tx_t tx);

/* Wait for outstanding work and free everything.  NULL is a no-op. */
int tx_destroy(rf_tx_t tx);

/* ============================================================ Autotuner
 *
 * The paper's handling thread tunes the GPU kernels at run time (Sec. III).
 * pfb_tune / ddc_tune time the candidate launch configurations of a handle
 * for buffers of `nsamples` samples on `hip_stream` -- frames per work-group
 * run and kernel variant for the PFB, persistent grid size for the DDC -- on
 * scratch buffers allocated and freed inside the call (the stream state is
 * not touched; the call waits for the handle's pending work first), keep the
 * fastest in the handle and append it to a text cache (RFCHAN_TUNE_CACHE, or
 * $HOME/.cache/rfchan_tune.txt).  *_apply_tuned loads a cached choice for a
 * buffer size (RF_EAGAIN if none is cached).  best_us (may be NULL) receives
 * the chosen configuration's time per launch. */
int pfb_tune(rf_pfb_t pfb, uint64_t nsamples, void *hip_stream, double *best_us);
int pfb_apply_tuned(rf_pfb_t pfb, uint64_t nsamples);
int pfb_tuned_config(rf_pfb_t pfb, int32_t *run_len, int32_t *variant);
int ddc_tune(rf_ddc_t ddc, uint64_t nsamples, void *hip_stream, double *best_us);
int ddc_apply_tuned(rf_ddc_t ddc, uint64_t nsamples);
int ddc_tuned_config(rf_ddc_t ddc, int32_t *grid);

/* ============================================================ Serving
 *
 * A server multiplexes many readout streams onto one GPU, the way the paper's
 * host threads hand pre-allocated buffers to the GPU signal-processing thread
 * through lock-free queues (Sec. III, Fig. 2).  Each stream is a PFB and/or a
 * DDC bank with its own filter history and oscillator phase kept on the
 * device.  Requests (one buffer of a stream each) are queued as they arrive; a
 * scheduler thread continuously forms batches from the oldest pending buffer
 * of every stream that has a free output slot, and runs each batch as grouped
 * kernels (one per PFB channel/tap class, one per DDC work-group size, which
 * follows the bank's tone count as in a single-stream launch) whose
 * work-groups stride over the buffers of all streams in the batch.  Requests
 * that arrive while a batch is on the GPU join the next one.  Streams are
 * admitted by their device-memory footprint against a budget.
 *
 * Input buffers are owned by the caller and kept alive until the request
 * completes.  They are device memory, or pinned host memory (hipHostMalloc)
 * for streams opened with host_slots > 0: the server copies such a buffer
 * into one of the stream's device staging slots on a copy stream of its own,
 * overlapped with the running batch, and the batch that uses it waits for
 * that copy only (the paper's host RAM -> GPU hop, Sec. II.B and Fig. 2).
 * Results stay in the stream's output slot until the caller releases it
 * (rfs_release).  All calls are thread-safe.
 */
typedef struct rfs_server *rfs_t;

#define RFS_PFB 1
#define RFS_DDC 2

#define RFS_MODE_SEQUENTIAL 0 /* one plain kernel per request, in arrival order (baseline) */
#define RFS_MODE_BATCHED 1    /* grouped persistent kernels, launched directly per batch */
#define RFS_MODE_GRAPH 2      /* grouped persistent kernels, replayed from prebuilt hipGraphs */

typedef struct {
    int32_t kinds;            /* RFS_PFB and/or RFS_DDC */
    int32_t nchan, ntaps;     /* PFB: N (power of two, 16..4096), M (1..16) */
    const float *proto;       /* PFB: host, N*M taps (copied) */
    int32_t ntones;           /* DDC: 1..65536 */
    const uint64_t *phase_inc;/* DDC: host, tuning words (copied) */
    const uint64_t *phase0;   /* DDC: host or NULL */
    int32_t lpf_taps;         /* DDC: T (1..4096) */
    const float *lpf;         /* DDC: host, T taps (copied) */
    int32_t decim;            /* DDC: D */
    uint64_t max_buffer;      /* largest nsamples of one request */
    int32_t out_slots;        /* output slots of the stream, >= 1 */
    int32_t host_slots;       /* device staging slots for pinned-host buffers
                                 (max_buffer samples each), 0 = device buffers only */
} rfs_stream_desc;

typedef struct {
    int32_t stream;
    int32_t slot;             /* output slot holding the results */
    uint64_t tag;             /* caller's tag from rfs_submit */
    uint64_t nsamples;
    int32_t status;           /* RF_OK, or the error of this request */
    int32_t pad;
    uint64_t pfb_frames;      /* frames written (PFB streams) */
    const float *pfb_out;     /* device: pfb_frames x N complex64 */
    uint64_t ddc_outputs;     /* outputs per tone written (DDC streams) */
    uint64_t ddc_ld;          /* row stride of ddc_out in complex values */
    const float *ddc_out;     /* device: ntones x ddc_ld complex64, tone-major */
    double t_submit, t_launch, t_done;  /* seconds on rfs_now()'s clock */
} rfs_completion;

typedef struct {
    uint64_t requests, batches, samples;
    uint64_t bytes_admitted, bytes_budget;
    int32_t streams_open, pad;
    double gpu_busy_seconds;  /* sum of batch durations (host-observed) */
} rfs_stats;

/* Create a server on the current device with a device-memory budget for
 * stream state and output slots, a scheduling mode (RFS_MODE_*) and a limit on
 * open streams.  Starts the scheduler thread. */
int rfs_create(rfs_t *out, uint64_t hbm_budget_bytes, int32_t mode, int32_t max_streams);

/* Device bytes a stream with this description occupies (state, output slots
 * and staging slots). */
uint64_t rfs_stream_footprint(const rfs_stream_desc *desc);

/* Open a stream; *id receives its number.  RF_EAGAIN when its footprint does
 * not fit in the remaining budget or max_streams are open (retry after others
 * close); RF_EINVAL for a bad description. */
int rfs_open_stream(rfs_t s, const rfs_stream_desc *desc, int32_t *id);

/* Queue the next buffer of stream `id` (nsamples <= max_buffer): a device
 * pointer, or a pinned-host pointer when the stream has host_slots.  RF_EINVAL
 * for pageable host memory, for a pinned-host pointer on a stream without
 * staging slots, or for a misaligned pointer. */
int rfs_submit(rfs_t s, int32_t id, const int16_t *iq, uint64_t nsamples, uint64_t tag);

/* Collect up to `max` completions, waiting up to timeout_us (0: do not wait). */
int rfs_poll(rfs_t s, rfs_completion *out, int32_t max, int32_t *count, int32_t timeout_us);

/* Return an output slot of stream `id` to the server after reading it. */
int rfs_release(rfs_t s, int32_t id, int32_t slot);

/* Close a stream with no queued or running requests (RF_EAGAIN otherwise). */
int rfs_close_stream(rfs_t s, int32_t id);

int rfs_get_stats(rfs_t s, rfs_stats *st);

/* The server's monotonic clock in seconds (for arrival timestamps). */
double rfs_now(void);

/* Stop the scheduler, wait for the GPU, free everything (NULL is accepted). */
int rfs_destroy(rfs_t s);

#ifdef __cplusplus
}
#endif

#endif /* RFCHAN_H */
