"""Seeded synthetic inputs for the readout channelizer and demodulator.

This module is shared by the FP64 oracle tests and the GPU path's tests and
benchmarks.  It holds only input recipes: filter designs handed to both sides
as data, tuning words, and int16 I/Q streams of tones plus Gaussian noise.
None of the channelizer's or demodulator's own arithmetic lives here.

Conventions (paper Sec. II.A: 14-bit ADC, 200 Ms/s complex baseband):

* A stream is interleaved int16 I/Q (I at even index, Q at odd), values
  rounded half-to-even and clipped to the 14-bit range [-8192, 8191].
* A tone is described by a 64-bit tuning word w: its phase at sample m is
  2 pi (w*m mod 2^64) / 2^64, i.e. frequency w / 2^64 * fs.  A bin-centred tone
  of an N-channel bank has w = k * 2^64 / N.
* Random draws follow one order: tone bins or tuning words, then phases
  U[0, 2 pi), then the noise, chunk by chunk (I then Q inside a chunk), from
  ``np.random.SeedSequence(seed)`` (tone parameters) and its children with
  ``spawn_key=(1, chunk)`` (noise of chunk ``chunk`` of 2^20 samples), so any
  sample range can be regenerated on its own.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

FS = 200e6                  # sample rate of the paper's SDR (Sec. II.A)
ADC_MIN, ADC_MAX = -8192, 8191
NOISE_CHUNK = 1 << 20       # samples per noise seed chunk
TWO64 = float(2 ** 64)

# --------------------------------------------------------------- windows


def window(name: str, L: int, beta: float = 9.0) -> np.ndarray:
    """Symmetric window of length L (denominator L-1)."""
    name = name.lower()
    if name == "hann":
        return np.hanning(L)
    if name == "hamming":
        return np.hamming(L)
    if name == "blackman":
        return np.blackman(L)
    if name == "kaiser":
        return np.kaiser(L, beta)
    if name in ("boxcar", "rect", "ones"):
        return np.ones(L)
    raise ValueError("unknown window %r" % name)


def pfb_prototype(N: int, M: int, win: str = "hann", beta: float = 9.0,
                  normalize: bool = True) -> np.ndarray:
    """Windowed-sinc prototype of length N*M (paper Sec. III.A).

    h[r] = w[r] * sinc((r - (L-1)/2) / N): the sinc's cut-off sits at half the
    channel spacing, so adjacent channels cross at about -6 dB.  Normalised to
    unit DC gain (sum h = 1) by default.
    """
    L = N * M
    r = np.arange(L, dtype=np.float64)
    h = window(win, L, beta) * np.sinc((r - (L - 1) / 2.0) / N)
    if normalize:
        h = h / h.sum()
    return h


def ddc_lowpass(T: int, fc: float, fs: float = FS, win: str = "blackman",
                beta: float = 9.0, normalize: bool = True) -> np.ndarray:
    """T-tap windowed-sinc low-pass with cut-off fc: w[k] sinc(2 fc/fs (k-(T-1)/2)), sum 1."""
    k = np.arange(T, dtype=np.float64)
    h = window(win, T, beta) * np.sinc(2.0 * fc / fs * (k - (T - 1) / 2.0))
    if normalize:
        h = h / h.sum()
    return h


def boxcar(D: int) -> np.ndarray:
    """The paper's moving-average anti-alias filter (Sec. III.B): h = 1/D, T = D."""
    return np.full(D, 1.0 / D)


# ----------------------------------------------------------- tuning words


def tuning_word(freq_hz: float, fs: float = FS) -> int:
    """round(f/fs * 2^64) mod 2^64 (negative frequencies wrap)."""
    return int(round(freq_hz / fs * TWO64)) % (1 << 64)


def bin_word(k: float, N: int) -> int:
    """Tuning word of (possibly fractional) bin k of an N-channel bank."""
    return int(round(k * TWO64 / N)) % (1 << 64)


def chirp_words(f0_hz: float, k_hz_per_s: float, fs: float = FS):
    """(inc, K) of the quadratic NCO for Eq. 1's phase 2 pi (f0 t + k t^2)
    sampled at t = m/fs: in cycles, f0 m/fs + k m^2/fs^2 = m (f0/fs + k/fs^2)
    + (2k/fs^2) m(m-1)/2, so inc = (f0/fs + k/fs^2) 2^64 and K = (2k/fs^2)
    2^64, each rounded to the nearest integer mod 2^64 (exact rational
    arithmetic on the given floats)."""
    from fractions import Fraction
    f0, k, fs_ = Fraction(f0_hz), Fraction(k_hz_per_s), Fraction(fs)
    inc = round((f0 / fs_ + k / fs_ ** 2) * (1 << 64)) % (1 << 64)
    K = round(2 * k / fs_ ** 2 * (1 << 64)) % (1 << 64)
    return int(inc), int(K)


def word_freq(w: int, fs: float = FS) -> float:
    """Frequency in Hz of tuning word w, in [-fs/2, fs/2)."""
    w = int(w) % (1 << 64)
    if w >= 1 << 63:
        w -= 1 << 64
    return w / TWO64 * fs


# ----------------------------------------------------------- quantisation


def quantize(x: np.ndarray) -> np.ndarray:
    """Complex samples -> interleaved int16 I/Q, rint (half-even) then clip to 14 bits."""
    x = np.asarray(x)
    out = np.empty(2 * x.size, dtype=np.int16)
    out[0::2] = np.clip(np.rint(x.real), ADC_MIN, ADC_MAX)
    out[1::2] = np.clip(np.rint(x.imag), ADC_MIN, ADC_MAX)
    return out


def iq_to_complex(iq: np.ndarray) -> np.ndarray:
    iq = np.asarray(iq).reshape(-1)
    return iq[0::2].astype(np.float64) + 1j * iq[1::2].astype(np.float64)


# ----------------------------------------------------------- tone streams


@dataclasses.dataclass
class ToneSet:
    words: np.ndarray      # uint64 tuning words
    amps: np.ndarray       # float64 amplitudes (LSB)
    phases: np.ndarray     # float64 initial phases (rad)


def _phase_angle(words: np.ndarray, m0: int) -> np.ndarray:
    """2 pi * ((w * m0) mod 2^64) / 2^64, from exact 64-bit integer products."""
    ph = words * np.uint64(m0 % (1 << 64))       # numpy uint64 wraps mod 2^64
    return ph.astype(np.float64) * (2.0 * np.pi / TWO64)


def tone_sum(tones: ToneSet, start: int, count: int, block: int = 1024,
             dtype=np.complex64) -> np.ndarray:
    """sum_t A_t exp(i(theta_t + 2 pi (w_t m mod 2^64)/2^64)) for m in [start, start+count).

    Evaluated blockwise as a matrix product: for m = m0 + k,
    exp(i phi(m0 + k)) = exp(i phi(m0)) exp(i phi(k)), with both phases taken
    from exact 64-bit integer products.
    """
    words = np.asarray(tones.words, dtype=np.uint64)
    nt = words.size
    out = np.zeros(count, dtype=np.complex128)
    if nt == 0 or count == 0:
        return out
    if nt <= 16:
        m = np.arange(start, start + count, dtype=np.uint64)
        for t in range(nt):
            ang = (m * words[t]).astype(np.float64) * (2.0 * np.pi / TWO64)
            out += tones.amps[t] * np.exp(1j * (ang + tones.phases[t]))
        return out
    k = np.arange(block, dtype=np.uint64)
    E = np.exp(1j * ((k[None, :] * words[:, None]).astype(np.float64)
                     * (2.0 * np.pi / TWO64))).astype(dtype)          # [nt, block]
    a_amp = np.asarray(tones.amps, dtype=np.float64)
    a_ph = np.asarray(tones.phases, dtype=np.float64)
    nblk = (count + block - 1) // block
    chunk_blocks = max(1, (1 << 22) // block)
    for b0 in range(0, nblk, chunk_blocks):
        b1 = min(nblk, b0 + chunk_blocks)
        m0 = start + np.arange(b0, b1, dtype=np.uint64) * np.uint64(block)
        ang = (m0[:, None] * words[None, :]).astype(np.float64) * (2.0 * np.pi / TWO64)
        A = (a_amp[None, :] * np.exp(1j * (ang + a_ph[None, :]))).astype(dtype)  # [nb, nt]
        seg = (A @ E).reshape(-1)
        lo = b0 * block
        hi = min(count, b1 * block)
        out[lo:hi] = seg[: hi - lo]
    return out


def noise(seed: int, sigma: float, start: int, count: int) -> np.ndarray:
    """Complex Gaussian noise, per-component sigma, seeded per 2^20-sample chunk."""
    out = np.empty(count, dtype=np.complex128)
    if sigma == 0 or count == 0:
        out[:] = 0
        return out
    c0 = start // NOISE_CHUNK
    c1 = (start + count - 1) // NOISE_CHUNK
    for c in range(c0, c1 + 1):
        rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(1, c)))
        re = rng.standard_normal(NOISE_CHUNK)
        im = rng.standard_normal(NOISE_CHUNK)
        lo = max(start, c * NOISE_CHUNK)
        hi = min(start + count, (c + 1) * NOISE_CHUNK)
        s = slice(lo - c * NOISE_CHUNK, hi - c * NOISE_CHUNK)
        out[lo - start: hi - start] = sigma * (re[s] + 1j * im[s])
    return out


@dataclasses.dataclass
class StreamSpec:
    seed: int
    tones: ToneSet
    sigma: float

    def complex(self, start: int, count: int) -> np.ndarray:
        return tone_sum(self.tones, start, count) + noise(self.seed, self.sigma, start, count)

    def iq(self, start: int, count: int) -> np.ndarray:
        """int16 interleaved I/Q for samples [start, start+count)."""
        return quantize(self.complex(start, count))


def random_phases(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.uniform(0.0, 2.0 * np.pi, n)


def random_words(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniform random 64-bit tuning words (uniform over the whole +-fs/2 band)."""
    return rng.integers(0, 1 << 64, size=n, dtype=np.uint64, endpoint=False)


# ------------------------------------------------------------ workloads


@dataclasses.dataclass
class PfbWorkload:
    name: str
    N: int
    M: int
    h: np.ndarray
    stream: StreamSpec
    nsamples: int
    buffer: int            # samples per process() call


@dataclasses.dataclass
class DdcWorkload:
    name: str
    words: np.ndarray      # NCO tuning words (uint64)
    phase0: np.ndarray     # NCO initial phases (uint64)
    h: np.ndarray
    D: int
    stream: StreamSpec
    nsamples: int
    buffer: int


def pfb_small(seed: int = 1, nsamples: int = 1 << 20) -> PfbWorkload:
    """PFB parity case: N=64, M=4, Hann-sinc prototype (L=256, unit DC gain).

    8 distinct random bin-centred tones (A = 2000 LSB, random phases) plus
    complex Gaussian noise with sigma = 1000 LSB per component; 2^20 samples
    give 16381 frames.
    """
    N, M = 64, 4
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    bins = rng.choice(N, size=8, replace=False)
    ph = random_phases(rng, 8)
    words = np.array([bin_word(int(b), N) for b in bins], dtype=np.uint64)
    tones = ToneSet(words, np.full(8, 2000.0), ph)
    return PfbWorkload("pfb N=64 M=4 hann", N, M, pfb_prototype(N, M, "hann"),
                       StreamSpec(seed, tones, 1000.0), nsamples, nsamples)


def pfb_production(seed: int = 2, nsamples: int = 1 << 28,
                   buffer: int = 1 << 24) -> PfbWorkload:
    """PFB production case: N=1024, M=8, Kaiser(beta=9)-sinc prototype (L=8192).

    1000 tones with uniform random 64-bit tuning words (the whole +-100 MHz band
    at 200 Ms/s), A = 8 LSB each, random phases, plus sigma = 200 LSB noise;
    2^28 samples streamed in 2^24-sample buffers.
    """
    N, M = 1024, 8
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    words = random_words(rng, 1000)
    ph = random_phases(rng, 1000)
    tones = ToneSet(words, np.full(1000, 8.0), ph)
    return PfbWorkload("pfb N=1024 M=8 kaiser9", N, M, pfb_prototype(N, M, "kaiser", 9.0),
                       StreamSpec(seed, tones, 200.0), nsamples, buffer)


def ddc_bank(seed: int = 3, ntones: int = 1000, nsamples: int = 1 << 27,
             buffer: int = 1 << 23, T: int = 1024, D: int = 1000,
             fc: float = 80e3) -> DdcWorkload:
    """DDC bank: 1000 NCO tones at uniform random 64-bit tuning words (non-grid).

    1024-tap Blackman-windowed sinc low-pass, cut-off 80 kHz at fs = 200 Ms/s,
    unit DC gain, decimation 1000; the input carries a tone of A = 8 LSB at
    every NCO frequency (random phase) plus sigma = 200 LSB noise; 2^27
    samples in 2^23-sample buffers, giving 134217 outputs per tone.
    """
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    words = random_words(rng, ntones)
    ph = random_phases(rng, ntones)
    tones = ToneSet(words, np.full(ntones, 8.0), ph)
    h = ddc_lowpass(T, fc, FS, "blackman")
    return DdcWorkload("ddc tones=%d T=%d D=%d blackman" % (ntones, T, D), words,
                       np.zeros(ntones, dtype=np.uint64), h, D,
                       StreamSpec(seed, tones, 200.0), nsamples, buffer)


def pfb_precision(seed: int = 4, nframes: int = 1 << 22) -> PfbWorkload:
    """Precision case: N=256, M=8, Kaiser(9); 128 bin-centred + 128 off-grid tones.

    Per-tone amplitude 2000*sqrt(8/256) LSB keeps the composite power of the
    8-tone parity case; sigma = 1000 LSB noise.
    """
    N, M = 256, 8
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    on = rng.choice(N, size=128, replace=False).astype(np.float64)
    off = rng.uniform(0.0, N, size=128)
    ph = random_phases(rng, 256)
    words = np.array([bin_word(float(k), N) for k in np.concatenate([on, off])],
                     dtype=np.uint64)
    tones = ToneSet(words, np.full(256, 2000.0 * np.sqrt(8.0 / 256.0)), ph)
    nsamples = (nframes - 1) * N + N * M
    return PfbWorkload("pfb N=256 M=8 kaiser9 precision", N, M,
                       pfb_prototype(N, M, "kaiser", 9.0),
                       StreamSpec(seed, tones, 1000.0), nsamples, nsamples)


def split_sizes(total: int, sizes: Sequence[int]) -> list:
    """Cut `total` samples into consecutive buffers following the pattern `sizes` (cycled)."""
    out, i, left = [], 0, total
    while left > 0:
        s = min(left, int(sizes[i % len(sizes)]))
        out.append(s)
        left -= s
        i += 1
    return out


# ------------------------------------------------- device-side generation
#
# The same recipe evaluated with torch on a GPU, for the full-size workloads
# (10^11 tone-sample terms are far too slow in numpy).  Tones: the blockwise
# matrix product of tone_sum() in FP32, from exact 64-bit integer phases.
# Noise: torch's normal generator seeded per 2^20-sample chunk, so any sample
# range can be regenerated; its random stream differs from the numpy
# backend's, the distribution is the same.


def _u64_angle_t(x):
    """int64 tensor holding uint64 phases -> angle 2 pi x / 2^64 (float64)."""
    import torch
    f = x.to(torch.float64)
    f = torch.where(f < 0, f + TWO64, f)
    return f * (2.0 * np.pi / TWO64)


def _noise_seed(seed: int, chunk: int) -> int:
    return (int(seed) * 1000003 + int(chunk) * 7919 + 12345) & 0x7FFFFFFFFFFFFFFF


def iq_torch(spec: StreamSpec, start: int, count: int, device="cuda", block: int = 1024):
    """int16 interleaved I/Q of samples [start, start+count) generated on `device`."""
    import torch
    dev = torch.device(device)
    out = torch.empty(2 * count, dtype=torch.int16, device=dev)
    if count == 0:
        return out
    words = torch.from_numpy(np.asarray(spec.tones.words, dtype=np.uint64).view(np.int64)).to(dev)
    amps = torch.from_numpy(np.asarray(spec.tones.amps, dtype=np.float64)).to(dev)
    phs = torch.from_numpy(np.asarray(spec.tones.phases, dtype=np.float64)).to(dev)
    nt = words.numel()
    k = torch.arange(block, dtype=torch.int64, device=dev)
    if nt:
        angk = _u64_angle_t(words[:, None] * k[None, :])                 # [nt, block]
        Er = torch.cos(angk).to(torch.float32).contiguous()
        Ei = torch.sin(angk).to(torch.float32).contiguous()
    c0 = start // NOISE_CHUNK
    c1 = (start + count - 1) // NOISE_CHUNK
    nb = NOISE_CHUNK // block
    for c in range(c0, c1 + 1):
        base = c * NOISE_CHUNK
        if nt:
            m0 = base + torch.arange(nb, dtype=torch.int64, device=dev) * block
            ang0 = _u64_angle_t(m0[:, None] * words[None, :]) + phs[None, :]   # [nb, nt]
            Ar = (amps[None, :] * torch.cos(ang0)).to(torch.float32).contiguous()
            Ai = (amps[None, :] * torch.sin(ang0)).to(torch.float32).contiguous()
            xr = (Ar @ Er - Ai @ Ei).reshape(-1)
            xi = (Ar @ Ei + Ai @ Er).reshape(-1)
        else:
            xr = torch.zeros(NOISE_CHUNK, dtype=torch.float32, device=dev)
            xi = torch.zeros(NOISE_CHUNK, dtype=torch.float32, device=dev)
        if spec.sigma:
            g = torch.Generator(device=dev)
            g.manual_seed(_noise_seed(spec.seed, c))
            nz = torch.randn(2, NOISE_CHUNK, generator=g, device=dev, dtype=torch.float32)
            xr = xr + spec.sigma * nz[0]
            xi = xi + spec.sigma * nz[1]
        lo = max(start, base)
        hi = min(start + count, base + NOISE_CHUNK)
        s = slice(lo - base, hi - base)
        q = torch.stack([xr[s], xi[s]], dim=1).round_().clamp_(ADC_MIN, ADC_MAX).to(torch.int16)
        out[2 * (lo - start): 2 * (hi - start)] = q.reshape(-1)
    return out
