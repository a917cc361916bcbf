"""The served multi-stream workload: stream descriptions, a Poisson arrival
schedule and a device-resident pool of synthetic int16 I/Q to slice buffers
from.

16 concurrent readout streams with channel counts drawn from {64, 256, 1024,
4096} and taps from {4, 8} (Kaiser(9)-sinc prototypes); half of them also run
a DDC bank of 10-2000 tones (log-uniform) with a 1024-tap Blackman-sinc
low-pass (80 kHz at 200 Ms/s) decimating by 1000.  Buffers of 2^U samples, U
uniform in 16..24, arrive per stream as a Poisson process with a mean rate of
100 Ms/s (1.6 Gs/s in total).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import (FS, StreamSpec, ToneSet, ddc_lowpass, iq_torch, pfb_prototype,
               random_words)


@dataclasses.dataclass
class StreamSpecMix:
    N: int
    M: int
    proto: np.ndarray
    ddc: Optional[tuple]          # (words, phase0, lpf, D) or None
    pool_offset: int              # first pool sample of this stream
    max_buffer: int


@dataclasses.dataclass
class Arrival:
    t: float                      # seconds from the start of the run
    stream: int
    nsamples: int
    pool_start: int               # pool sample where this buffer starts


def build_mix(seed: int = 5, nstreams: int = 16, duration_s: float = 10.0,
              rate_per_stream: float = 100e6, pool_samples: int = 1 << 28,
              umin: int = 16, umax: int = 24):
    """Stream descriptions and a merged arrival schedule (sorted by time)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    specs: List[StreamSpecMix] = []
    mean_buf = np.mean([2.0 ** u for u in range(umin, umax + 1)])
    for s in range(nstreams):
        N = int(rng.choice([64, 256, 1024, 4096]))
        M = int(rng.choice([4, 8]))
        ddc = None
        if s % 2 == 1:
            ntones = int(round(np.exp(rng.uniform(np.log(10), np.log(2000)))))
            words = random_words(rng, ntones)
            ddc = (words, None, ddc_lowpass(1024, 80e3, FS, "blackman"), 1000)
        specs.append(StreamSpecMix(N, M, pfb_prototype(N, M, "kaiser", 9.0), ddc,
                                   int(rng.integers(0, pool_samples // 2)), 1 << umax))
    arrivals: List[Arrival] = []
    for s, sp in enumerate(specs):
        t, pos = 0.0, sp.pool_offset
        while True:
            t += rng.exponential(mean_buf / rate_per_stream)
            if t >= duration_s:
                break
            n = int(2 ** rng.integers(umin, umax + 1))
            if pos + n > pool_samples:
                pos = 0
            arrivals.append(Arrival(t, s, n, pos))
            pos += n
    arrivals.sort(key=lambda a: a.t)
    return specs, arrivals


def make_pool(pool_samples: int = 1 << 28, seed: int = 5, device="cuda"):
    """Device-resident int16 I/Q pool: 64 random tones (A = 50 LSB) + sigma = 300 LSB noise."""
    rng = np.random.default_rng(np.random.SeedSequence(seed + 1000))
    tones = ToneSet(random_words(rng, 64), np.full(64, 50.0),
                           rng.uniform(0, 2 * np.pi, 64))
    return iq_torch(StreamSpec(seed + 1000, tones, 300.0), 0, pool_samples, device)
