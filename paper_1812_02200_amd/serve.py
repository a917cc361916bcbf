"""Multi-stream serving driver: Poisson arrivals onto the C++ serving core.

The readout-stream mix: 16 concurrent streams with channel counts drawn from
{64, 256, 1024, 4096} and taps from {4, 8} (Kaiser(9)-sinc prototypes); half of
them also run a DDC bank of 10-2000 tones (log-uniform) with a 1024-tap
Blackman-sinc low-pass (80 kHz at 200 Ms/s) decimating by 1000.  Buffers of
2^U samples, U uniform in 16..24, arrive per stream as a Poisson process with
a mean rate of 100 Ms/s (1.6 Gs/s in total).  Their content is sliced from a
pool of synthetic int16 I/Q (tones + noise) resident in device memory.

This module only schedules submissions and collects completions; every
sample is processed by the library's kernels.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Dict, List, Optional

import numpy as np

from . import _lib


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
    import siggen
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    specs: List[StreamSpecMix] = []
    mean_buf = np.mean([2.0 ** u for u in range(umin, umax + 1)])
    for s in range(nstreams):
        N = int(rng.choice([64, 256, 1024, 4096]))
        M = int(rng.choice([4, 8]))
        ddc = None
        if s % 2 == 1:
            ntones = int(round(np.exp(rng.uniform(np.log(10), np.log(2000)))))
            words = siggen.random_words(rng, ntones)
            ddc = (words, None, siggen.ddc_lowpass(1024, 80e3, siggen.FS, "blackman"), 1000)
        specs.append(StreamSpecMix(N, M, siggen.pfb_prototype(N, M, "kaiser", 9.0), ddc,
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
    import siggen
    rng = np.random.default_rng(np.random.SeedSequence(seed + 1000))
    tones = siggen.ToneSet(siggen.random_words(rng, 64), np.full(64, 50.0),
                           rng.uniform(0, 2 * np.pi, 64))
    return siggen.iq_torch(siggen.StreamSpec(seed + 1000, tones, 300.0), 0, pool_samples, device)


def run(specs, arrivals, pool, mode: int, budget: int = 48 << 30, realtime: bool = True,
        collect: bool = False, out_slots: int = 3, max_streams: int = 64) -> Dict:
    """Open the streams on a fresh server, replay the arrivals and collect completions.

    realtime: submit each buffer at its arrival time (latency run); otherwise
    submit everything at once (saturation run).  collect: copy every output to
    the host (for parity checks) before releasing its slot.
    """
    import torch
    srv = _lib.Server(budget, mode, max_streams)
    ids = []
    for sp in specs:
        desc, keep = _lib.Server.make_desc(
            pfb=(sp.N, sp.M, sp.proto), ddc=sp.ddc, max_buffer=sp.max_buffer, out_slots=out_slots)
        ids.append(srv.open_stream(desc, keep))
    base = pool.data_ptr()
    lat, outputs = [], {}
    done = 0
    total = len(arrivals)
    i = 0
    t0 = _lib.Server.now()
    first_submit = None

    def drain(timeout_us):
        nonlocal done
        for c in srv.poll(256, timeout_us):
            if c["status"] != 0:
                raise RuntimeError("request failed with status %d" % c["status"])
            lat.append((c["t_done"] - c["t_submit"], c["t_done"]))
            if collect:
                s = ids.index(c["stream"])
                rec = {}
                if c["pfb_frames"]:
                    n = c["pfb_frames"] * specs[s].N
                    t = torch.empty(n, dtype=torch.complex64, device="cuda")
                    _copy_dev(t, c["pfb_out"], n * 8)
                    rec["pfb"] = t.view(-1, specs[s].N).cpu().numpy()
                else:
                    rec["pfb"] = np.zeros((0, specs[s].N), np.complex64)
                if specs[s].ddc is not None:
                    nt = len(specs[s].ddc[0])
                    ld = c["ddc_ld"]
                    t = torch.empty(nt * ld, dtype=torch.complex64, device="cuda")
                    _copy_dev(t, c["ddc_out"], nt * ld * 8)
                    rec["ddc"] = t.view(nt, ld)[:, : c["ddc_outputs"]].cpu().numpy()
                outputs.setdefault(s, []).append((c["tag"], rec))
            srv.release(c["stream"], c["slot"])
            done += 1

    while done < total:
        now = _lib.Server.now() - t0
        while i < total and (not realtime or arrivals[i].t <= now):
            a = arrivals[i]
            if first_submit is None:
                first_submit = _lib.Server.now()
            srv.submit(ids[a.stream], base + 4 * a.pool_start, a.nsamples, i)
            i += 1
        if i < total and realtime:
            wait_us = int(max(0.0, (arrivals[i].t - (_lib.Server.now() - t0))) * 1e6)
            drain(min(wait_us, 2000))
        else:
            drain(2000)
    t_end = max(t for _, t in lat) if lat else _lib.Server.now()
    stats = srv.stats()
    srv.close()
    lat_ms = np.array([l for l, _ in lat]) * 1e3
    samples = sum(a.nsamples for a in arrivals)
    span = t_end - (first_submit if first_submit else t0)
    res = {
        "requests": total, "samples": samples, "seconds": span,
        "msamples_per_s": samples / span / 1e6 if span > 0 else 0.0,
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "max": float(lat_ms.max()), "mean": float(lat_ms.mean())},
        "batches": stats["batches"], "gpu_busy_seconds": stats["gpu_busy_seconds"],
    }
    if collect:
        res["outputs"] = {s: [r for _, r in sorted(v, key=lambda x: x[0])] for s, v in outputs.items()}
    return res


def _copy_dev(dst_tensor, src_ptr: int, nbytes: int) -> None:
    """Device-to-device copy of a completion's output (torch owns the destination)."""
    import ctypes

    import torch
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    torch.cuda.synchronize()
    rc = hip.hipMemcpy(dst_tensor.data_ptr(), src_ptr, nbytes, 3)   # device to device
    if rc != 0:
        raise RuntimeError("hipMemcpy failed (%d)" % rc)
