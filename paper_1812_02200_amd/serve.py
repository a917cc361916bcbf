"""Replay of an arrival schedule onto the C++ serving core (rfs_* calls).

`run` opens one server stream per stream description, submits each buffer at
its arrival time (or all at once for a saturation run) and collects the
completions with their latencies.  A stream description needs N, M, proto,
ddc ((words, phase0, lpf, D) or None) and max_buffer; an arrival needs t,
stream, nsamples and pool_start (a sample offset into `pool`, a device or
pinned-host int16 I/Q tensor).  This module only schedules submissions and
collects completions; every sample is processed by the library's kernels.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from . import _lib


def run(specs, arrivals, pool, mode: int, budget: int = 48 << 30, realtime: bool = True,
        collect: bool = False, out_slots: int = 3, max_streams: int = 64, host_slots: int = 0) -> Dict:
    """Open the streams on a fresh server, replay the arrivals and collect completions.

    realtime: submit each buffer at its arrival time (latency run); otherwise
    submit everything at once (saturation run).  collect: copy every output to
    the host (for parity checks) before releasing its slot.  host_slots: staging
    slots per stream, needed when `pool` is pinned host memory.
    """
    import torch
    srv = _lib.Server(budget, mode, max_streams)
    ids = []
    for sp in specs:
        desc, keep = _lib.Server.make_desc(
            pfb=(sp.N, sp.M, sp.proto), ddc=sp.ddc, max_buffer=sp.max_buffer, out_slots=out_slots,
            host_slots=host_slots)
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
