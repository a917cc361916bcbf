#!/usr/bin/env python3
"""Benchmark of the readout hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload all|pfb|ddc]

One step is one pass of the hot path over one batch of synthetic input:
  * PFB: N=1024 channels, M=8 taps, Kaiser(9)-sinc prototype, 2^28 int16 I/Q
    samples in 16 buffers of 2^24 (one pfb_process call per buffer), FIR
    history carried across buffers and steps (a continuous stream);
  * DDC: 1000 tones, 1024-tap Blackman-sinc low-pass, decimation 1000, 2^27
    samples in 16 buffers of 2^23, NCO phase and FIR history carried.
Inputs are generated on the device before timing and stay resident in HBM.
`value` is the PFB's sustained input rate (Msamples/s); the DDC's figures are
in the "ddc" object.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TF = 157.3    # MI355X FP32 vector, published (packed FP32 included)
# The kernels are built without packed FP32 (two-lane v_pk_* forms), so the
# FP32 FMA ceiling they can reach is half of that: 256 CUs x 4 SIMDs x 16 lanes
# x 2 flop x 2.4 GHz.  VALU issue: 256 x 4 x 16 x 2.4e9 lane-instructions/s.
FP32_FMA_PEAK_TF = 78.6
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hbm_traffic_pfb_n1024_m8_ddc_1000tones.md")
TRACE_PROFILE = os.path.join(ROOT, "profiles", "kernel_trace_pfb_n1024_m8_ddc_1000tones_bench.md")
MFMA_PROFILE = os.path.join(ROOT, "profiles", "mfma_busy_precision_n256_m8.md")
KERNEL_SOURCES = os.path.join(ROOT, "paper_1812_02200_amd", "csrc")
METRIC = "sustained Msamples/s (N=1024 PFB, 1000-tone DDC) + p99 buffer latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="all",
                    help="comma-separated legs: all, pfb, ddc, tx, large, precision, serving, copyprobe")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate CPU time budget per oracle baseline sample")
    ap.add_argument("--pfb-shape", default=None, metavar="RUN_LEN:VARIANT",
                    help="use this PFB launch shape instead of autotuning (to profile the shape a "
                         "timed run chose)")
    ap.add_argument("--ddc-grid", type=int, default=None,
                    help="use this DDC grid instead of autotuning")
    ap.add_argument("--trace-summary", metavar="DIR",
                    help="summarise a rocprofv3 --kernel-trace run of this script (the library's "
                         "kernels) as markdown, and exit")
    ap.add_argument("--bench-out", metavar="FILE",
                    help="with --trace-summary: the profiled run's own output (its JSON line)")
    ap.add_argument("--mfma-summary", metavar="DIR",
                    help="summarise a rocprofv3 --pmc run (MFMA counters) of --workload precision, and exit")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "PROBE_FETCH_DIR",
                                                       "PROBE_WRITE_DIR"),
                    help="summarise rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this script "
                         "(bench workloads, then --workload copyprobe) as markdown, and exit")
    return ap.parse_args()


# ------------------------------------------------------- HBM traffic (PMC)

# The sources the profiled kernels (the timed PFB and DDC kernels, the MFMA
# DFT of the precision leg) are compiled from, with their launch code.
PROFILED_SOURCES = ("fft_device.hpp", "rf_internal.hpp", "pfb_kernels.hpp", "pfb_launch.hip", "pfb_n1024.hip",
                    "ddc_kernels.hip", "pfb_mfma.hpp", "pfb_mfma.hip", "pfb_mfma_n256.hip")


def sources_digest():
    """SHA-256 over the profiled kernels' sources: counters and traces taken on
    other sources are stale."""
    h = hashlib.sha256()
    for name in sorted(PROFILED_SOURCES):
        h.update(name.encode())
        with open(os.path.join(KERNEL_SOURCES, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when there is none or the kernel sources changed since it was taken."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            for line in fh:
                if line.startswith("traffic-json: "):
                    rec = json.loads(line[len("traffic-json: "):])
                    if rec.get("sources_sha256") != sources_digest():
                        return None
                    k = rec.get("kernels", {}).get(kernel)
                    return None if k is None else float(k["hbm_bytes_per_launch"])
    except OSError:
        return None
    return None


def _profile_json(path, tag):
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith(tag):
                    rec = json.loads(line[len(tag):])
                    return rec if rec.get("sources_sha256") == sources_digest() else None
    except OSError:
        return None
    return None


def profiled_trace(kernel):
    """The committed kernel trace's record of the timed launches of `kernel`
    (average duration in that profiled run, and that run's own event timing),
    or None when there is none or the kernel sources changed since."""
    rec = _profile_json(TRACE_PROFILE, "trace-json: ")
    return None if rec is None else rec.get("kernels", {}).get(kernel)


def profiled_mfma():
    rec = _profile_json(MFMA_PROFILE, "mfma-json: ")
    return None if rec is None else rec.get("kernels")


SHAPES = {}                    # launch shapes given on the command line (no autotuning)

COPY_PROBE_ELEMS = 1 << 26     # int32 elements per probe copy: 256 MiB read, 256 MiB written


def bench_copyprobe(torch):
    """A plain elementwise copy (torch.neg on int32) of known size, to calibrate
    the FETCH_SIZE / WRITE_SIZE counters."""
    src = torch.randint(-1000, 1000, (COPY_PROBE_ELEMS,), dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return {"copyprobe": {"bytes_read": 4 * COPY_PROBE_ELEMS, "bytes_written": 4 * COPY_PROBE_ELEMS,
                          "launches": 5}}


def _pmc_rows(d):
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, match):
    """{(kernel, grid): [counter value per dispatch]} for kernels whose name contains `match`."""
    out = {}
    for r in rows:
        if match in r["Kernel_Name"]:
            out.setdefault((r["Kernel_Name"].split("(")[0], int(r["Grid_Size"])), []).append(
                float(r["Counter_Value"]))
    return out


def _trace_rows(d):
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        with open(f) as fh:
            rows += [r for r in csv.DictReader(fh) if "rfk::" in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    return rows


def _bench_line(path):
    """The JSON line a profiled bench.py run printed (its own event timing)."""
    if not path:
        return None
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{") and '"metric"' in line:
                return json.loads(line)
    return None


def trace_summary(d, bench_out=None):
    """Markdown summary of a rocprofv3 --kernel-trace run of this script, plus a
    trace-json line: for the PFB and DDC legs, the average duration of exactly
    the timed launches (the last steps x buffers dispatches of the timed kernel
    before the next leg's kernels), beside the same run's event timing."""
    rows = _trace_rows(d)
    stats = {}
    for r in rows:
        name = r["Kernel_Name"].replace("void ", "").split("(")[0]
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        stats.setdefault(name, []).append(dur)
    print("| kernel | calls | average us | min us | max us |")
    print("|---|---|---|---|---|")
    for name, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        print("| `%s` | %d | %.1f | %.1f | %.1f |" % (name, len(v), np.mean(v), min(v), max(v)))
    line = _bench_line(bench_out)
    rec = {"sources_sha256": sources_digest(), "kernels": {}}
    if line:
        for leg, key, kern_us in (("pfb", "pfb_fir_fft", (line.get("pfb") or {}).get("kernel_us")),
                                  ("ddc", "ddc_bank", (line.get("ddc") or {}).get("kernel_us"))):
            leg_rec = line.get(leg) if leg != "pfb" else line.get("pfb")
            if not leg_rec or kern_us is None:
                continue
            n_timed = int(line["steps"]) * (16 if leg == "pfb" else 16)
            shape = leg_rec.get("tuned", {})
            # the timed kernel: the most frequent instance of this family in
            # the trace's longest run of back-to-back identical dispatches
            fam = [i for i, r in enumerate(rows) if key in r["Kernel_Name"]]
            best, cur, best_end = 0, 0, -1
            for j, i in enumerate(fam):
                if j and rows[i]["Kernel_Name"] == rows[fam[j - 1]]["Kernel_Name"] and \
                        rows[i]["Grid_Size_X"] == rows[fam[j - 1]]["Grid_Size_X"] and i == fam[j - 1] + 1:
                    cur += 1
                else:
                    cur = 1
                if cur >= best:
                    best, best_end = cur, j
            timed = [rows[fam[j]] for j in range(best_end - n_timed + 1, best_end + 1)] if best >= n_timed else []
            if not timed:
                continue
            durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in timed]
            span = (int(timed[-1]["End_Timestamp"]) - int(timed[0]["Start_Timestamp"])) / 1e3 / len(timed)
            rec["kernels"][key] = {"kernel": timed[0]["Kernel_Name"].replace("void ", "").split("(")[0],
                                   "grid": int(timed[0]["Grid_Size_X"]), "timed_launches": len(timed),
                                   "avg_us": float(np.mean(durs)), "min_us": float(min(durs)),
                                   "max_us": float(max(durs)), "span_us_per_launch": span,
                                   "event_us_per_launch": float(kern_us), "shape": shape}
        rec["bench_value"] = line.get("value")
        rec["device"] = line.get("device")
    print()
    for key, k in rec["kernels"].items():
        print("Timed launches of `%s` (grid %d threads): %d, trace average %.2f us (min %.2f, max %.2f), "
              "first start to last end %.2f us per launch; the same run's HIP-event timing %.2f us per launch."
              % (k["kernel"], k["grid"], k["timed_launches"], k["avg_us"], k["min_us"], k["max_us"],
                 k["span_us_per_launch"], k["event_us_per_launch"]))
    print()
    print("trace-json: " + json.dumps(rec))


def mfma_summary(d):
    """MFMA activity of the precision leg's kernels from a rocprofv3 --pmc run
    (SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE, SQ_INSTS_VALU_MFMA_MOPS_F16 /
    _BF16): busy fraction = busy cycles summed over the SIMDs / (cycles of
    one XCD x SIMDs), GRBM_GUI_ACTIVE being summed over the 8 XCDs."""
    rows = _pmc_rows(d)
    per = {}
    for r in rows:
        if "mfma" not in r["Kernel_Name"]:
            continue
        k = (r["Kernel_Name"].replace("void ", "").split("(")[0], r["Dispatch_Id"])
        per.setdefault(k, {})[r["Counter_Name"]] = float(r["Counter_Value"])
    by_kernel = {}
    for (name, _), c in per.items():
        by_kernel.setdefault(name, []).append(c)
    simds = 256 * 4
    rec = {"sources_sha256": sources_digest(), "kernels": {}}
    print("| kernel | dispatches | MFMA busy cycles (sum of SIMDs) | GPU cycles per XCD | MFMA busy fraction | MFMA ops (MOPS counter) |")
    print("|---|---|---|---|---|---|")
    for name, cs in sorted(by_kernel.items()):
        busy = np.median([c.get("SQ_VALU_MFMA_BUSY_CYCLES", np.nan) for c in cs])
        gui = np.median([c.get("GRBM_GUI_ACTIVE", np.nan) for c in cs]) / 8.0
        mops = np.median([c.get("SQ_INSTS_VALU_MFMA_MOPS_F16", 0.0) + c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)
                          for c in cs])
        frac = busy / (gui * simds) if gui > 0 else float("nan")
        rec["kernels"][name] = {"dispatches": len(cs), "mfma_busy_cycles": busy, "cycles_per_xcd": gui,
                                "mfma_busy_frac": frac, "mfma_mops": mops}
        print("| `%s` | %d | %.4g | %.4g | %.3f | %.4g |" % (name, len(cs), busy, gui, frac, mops))
    print()
    print("mfma-json: " + json.dumps(rec))


def pmc_summary(fetch_dir, write_dir, pf_dir, pw_dir):
    fr, wr, pfr, pwr = (_pmc_rows(d) for d in (fetch_dir, write_dir, pf_dir, pw_dir))
    # calibration: the copy probe's five torch.neg dispatches are its last ones
    def last5(rows):
        rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
        return [float(r["Counter_Value"]) for r in rows[-5:]]
    pf, pw = last5(pfr), last5(pwr)
    want = 4.0 * COPY_PROBE_ELEMS / 1024.0          # KiB read = KiB written per probe launch
    f_scale = want / np.median(pf)
    w_scale = want / np.median(pw)
    lines = ["| kernel | grid (threads) | launches | FETCH_SIZE KiB/launch | WRITE_SIZE KiB/launch |"
             " HBM bytes/launch (scaled) | algorithmic bytes/launch | ratio |",
             "|---|---|---|---|---|---|---|---|"]
    alg = {"pfb_fir_fft": 12.0 * (1 << 24), "ddc_bank": None}
    kern = {}
    for name in ("pfb_fir_fft", "ddc_bank"):
        fd, wd = _per_dispatch(fr, name), _per_dispatch(wr, name)
        if not fd or not wd:
            continue
        # the timed launches are the most frequent shape (the tuner's trials are few each)
        key = max(fd, key=lambda k: len(fd[k]))
        fk, wk = float(np.median(fd[key])), float(np.median(wd.get(key, [np.nan])))
        hbm = fk * 1024 * f_scale + wk * 1024 * w_scale
        a = alg[name]
        if name == "ddc_bank":
            # 2^23 input samples (4 B) + 1000 tones x 8388.6 outputs (8 B) per launch
            a = 4.0 * (1 << 23) + 8.0 * 1000 * ((1 << 23) / 1000.0)
        kern[name] = {"grid": key[1], "launches": len(fd[key]), "fetch_kib": fk, "write_kib": wk,
                      "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": a}
        lines.append("| %s | %d | %d | %.1f | %.1f | %.4g | %.4g | %.3f |"
                     % (name, key[1], len(fd[key]), fk, wk, hbm, a, hbm / a))
    rec = {"sources_sha256": sources_digest(), "fetch_scale": f_scale, "write_scale": w_scale,
           "kernels": kern}
    print("Counter scale factors from the copy probe (torch.neg over %d int32, %.0f KiB read and "
          "written per launch): FETCH_SIZE x %.3f, WRITE_SIZE x %.3f (medians %.1f / %.1f KiB)."
          % (COPY_PROBE_ELEMS, want, f_scale, w_scale, np.median(pf), np.median(pw)))
    print()
    print("\n".join(lines))
    print()
    print("traffic-json: " + json.dumps(rec))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ------------------------------------------------------------------ PFB

def bench_pfb(rf, torch, siggen, steps, warmup):
    w = siggen.pfb_production()
    log("pfb: generating %d samples on the device" % w.nsamples)
    d = siggen.iq_torch(w.stream, 0, w.nsamples)
    nbuf = w.nsamples // w.buffer
    fpb = w.buffer // w.N                           # frames per buffer in steady state
    out = torch.empty((nbuf, fpb, w.N), dtype=torch.complex64, device="cuda")
    if SHAPES.get("pfb"):
        os.environ["RFCHAN_PFB_RUN_LEN"], os.environ["RFCHAN_PFB_VARIANT"] = SHAPES["pfb"].split(":")
    p = rf.Pfb(w.N, w.M, w.h, max_samples_per_call=w.buffer)
    os.environ.pop("RFCHAN_PFB_RUN_LEN", None)     # this handle only
    os.environ.pop("RFCHAN_PFB_VARIANT", None)
    if SHAPES.get("pfb"):
        rl, var = p.tuned_config()
        tuned = (float("nan"), rl, var)
    else:
        tuned = p.tune(w.buffer)      # launch shape chosen by the autotuner (setup, untimed)
    log("pfb shape: %.1f us/launch (tuner), run_len=%d variant=%d" % tuned)
    s = torch.cuda.current_stream()
    sh = s.cuda_stream
    base_in, base_out = d.data_ptr(), out.data_ptr()
    frames = [0]

    def step():
        for b in range(nbuf):
            frames[0] += p.process_ptr(base_in + 4 * b * w.buffer, w.buffer,
                                       base_out + 8 * b * fpb * w.N, fpb, sh)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    f0 = frames[0]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        step()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    launches = steps * nbuf
    samples = steps * w.nsamples
    kern_s = ms / 1e3 / launches
    bytes_per_launch = 12.0 * w.buffer                  # 4 B in + 8 B out per sample
    achieved = bytes_per_launch / kern_s / 1e9
    # the same stream returning 16 chosen channels instead of all 1024
    ch = np.random.default_rng(21).permutation(w.N)[:16].astype(np.int32)
    p.set_channels(ch)
    sub = torch.empty((nbuf, fpb, ch.size), dtype=torch.complex64, device="cuda")

    def sstep():
        for b in range(nbuf):
            p.process_ptr(base_in + 4 * b * w.buffer, w.buffer, sub.data_ptr() + 8 * b * fpb * ch.size, fpb, sh)

    sstep()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        sstep()
    e1.record(s)
    torch.cuda.synchronize()
    sms = e0.elapsed_time(e1)
    p.set_channels(None)
    res = {
        "value": samples / (ms / 1e3) / 1e6,
        "ms_per_step": ms / steps,
        "wall_ms_per_step": wall * 1e3 / steps,
        "chosen_16_channels": {"value": samples / (sms / 1e3) / 1e6, "unit": "Msamples/s",
                               "kernel_us": sms * 1e3 / launches,
                               "hbm_gbs": (4.0 + 8.0 * 16 / w.N) * w.buffer / (sms / 1e3 / launches) / 1e9},
        "frames_per_step": (frames[0] - f0) / steps,
        "kernel_us": kern_s * 1e6,
        "tuned": {"run_len": tuned[1], "variant": tuned[2], "us_per_launch": tuned[0]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic("pfb_fir_fft"),
                     "trace": _trace_frac("pfb_fir_fft", bytes_per_launch, HBM_PEAK_GBS * 1e9),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-probe scaled)",
                     "per_launch": "12 B x 2^24 samples = %.1f MB" % (bytes_per_launch / 1e6)},
        "config": {"workload": w.name + ", 2^28 int16 I/Q samples in 2^24-sample buffers",
                   "N": w.N, "M": w.M, "buffer_samples": w.buffer, "samples_per_step": w.nsamples},
    }
    return res, (w, d)


def _trace_frac(kernel, units_per_launch, peak_per_s):
    """The committed kernel trace of the timed launches (a profiled run of this
    script on an earlier box): its average duration, the roofline fraction it
    gives, and that run's own event timing; None if the sources changed."""
    t = profiled_trace(kernel)
    if not t:
        return None
    return {"avg_us": t["avg_us"], "frac": units_per_launch / (t["avg_us"] * 1e-6) / peak_per_s,
            "event_us_same_run": t["event_us_per_launch"], "launches": t["timed_launches"],
            "source": os.path.relpath(TRACE_PROFILE, ROOT)}


def cpu_model():
    """The host CPU's model name (first processor entry), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def cpu_pfb(oracle, w, d, budget_s):
    """The FP64 oracle on the same stream (host cores), repeated up to ~budget_s,
    then on one thread over a leading part of the frames (~budget_s / 2)."""
    nf = oracle.pfb_nframes(w.nsamples, w.N, w.M)
    iq = d.cpu().numpy()
    frames = np.arange(nf)
    reps, t = 0, 0.0
    while t < budget_s and reps < 64:
        t0 = time.perf_counter()
        oracle.pfb(w.h, w.N, w.M, iq=iq, frames=frames)
        t += time.perf_counter() - t0
        reps += 1
    cores = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        k = 256
        t0 = time.perf_counter()
        oracle.pfb(w.h, w.N, w.M, iq=iq, frames=np.arange(k))
        t1 = time.perf_counter() - t0
        k = int(min(nf, max(k, k * 0.5 * budget_s / max(t1, 1e-6))))
        t0 = time.perf_counter()
        oracle.pfb(w.h, w.N, w.M, iq=iq, frames=np.arange(k))
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_num_threads(cores)
    return {"value": reps * nf * w.N / t / 1e6, "unit": "Msamples/s", "cores": cores,
            "kind": "oracle", "seconds": t, "cpu_model": cpu_model(),
            "sample": "all %d frames of the 2^28-sample N=1024 M=8 stream x %d passes, FP64, "
                      "OpenMP over frames" % (nf, reps),
            "single_thread": {"value": k * w.N / t1 / 1e6, "unit": "Msamples/s", "cores": 1, "seconds": t1,
                              "sample": "the first %d frames of the same stream, FP64, one thread" % k}}


# ------------------------------------------------------------------ DDC

def bench_ddc(rf, torch, siggen, steps, warmup):
    w = siggen.ddc_bank()
    log("ddc: generating %d samples on the device" % w.nsamples)
    d = siggen.iq_torch(w.stream, 0, w.nsamples)
    nbuf = w.nsamples // w.buffer
    ld = w.buffer // w.D + 2
    out = torch.empty((nbuf, w.words.size, ld), dtype=torch.complex64, device="cuda")
    if SHAPES.get("ddc"):
        os.environ["RFCHAN_DDC_GRID"] = str(SHAPES["ddc"])
    dd = rf.Ddc(w.words, w.h, w.D, w.phase0, max_samples_per_call=w.buffer)
    os.environ.pop("RFCHAN_DDC_GRID", None)        # this handle only
    dtuned = (float("nan"), dd.tuned_config()) if SHAPES.get("ddc") else dd.tune(w.buffer)
    log("ddc tuned: %.1f us/launch, grid=%d" % dtuned)
    s = torch.cuda.current_stream()
    sh = s.cuda_stream
    base_in, base_out = d.data_ptr(), out.data_ptr()
    nout = [0]

    def step():
        for b in range(nbuf):
            nout[0] += dd.process_ptr(base_in + 4 * b * w.buffer, w.buffer,
                                      base_out + 8 * b * w.words.size * ld, ld, sh)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    n0 = nout[0]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        step()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    outs = (nout[0] - n0)
    launches = steps * nbuf
    kern_s = ms / 1e3 / launches
    flop = 8.0 * w.h.size * w.words.size * outs / launches    # one complex MAC per tap-tone
    achieved = flop / kern_s / 1e12
    # VALU issue: 9 instructions per sample-tone (64-bit phase step, two table
    # and copy addresses, four FMAs) against the chip's lane-instruction rate
    valu = 9.0 * w.h.size * w.words.size * outs / launches / kern_s
    # the same bank with chirped tones (Eq. 1 words; second-order accumulator)
    crng = np.random.default_rng(33)
    cinc, cK = [], []
    for _ in range(w.words.size):
        a_, b_ = siggen.chirp_words(float(crng.uniform(-90e6, 90e6)), float(crng.uniform(-2e13, 2e13)))
        cinc.append(a_)
        cK.append(b_)
    dc = rf.Ddc(np.array(cinc, np.uint64), w.h, w.D, w.phase0, max_samples_per_call=w.buffer,
                chirp=np.array(cK, np.uint64))
    dc.tune(w.buffer)

    def cstep():
        for b in range(nbuf):
            dc.process_ptr(base_in + 4 * b * w.buffer, w.buffer, base_out + 8 * b * w.words.size * ld, ld, sh)

    cstep()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        cstep()
    e1.record(s)
    torch.cuda.synchronize()
    cms = e0.elapsed_time(e1)
    dc.close()
    return {
        "value": steps * w.nsamples / (ms / 1e3) / 1e6,
        "unit": "Msamples/s",
        "ms_per_step": ms / steps,
        "kernel_us": kern_s * 1e6,
        "chirped": {"value": steps * w.nsamples / (cms / 1e3) / 1e6, "unit": "Msamples/s",
                    "kernel_us": cms * 1e3 / launches,
                    "workload": "the same bank with 1000 chirped tones (Eq. 1, |k| <= 2e13 Hz/s)"},
        "outputs_per_tone_per_step": outs / steps,
        "tuned": {"grid": dtuned[1], "us_per_launch": dtuned[0]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_FMA_PEAK_TF,
                     "unit": "TFLOP/s", "frac": achieved / FP32_FMA_PEAK_TF,
                     "traffic": profiled_traffic("ddc_bank"),
                     "trace": _trace_frac("ddc_bank", flop, FP32_FMA_PEAK_TF * 1e12),
                     "traffic_unit": "HBM bytes per launch",
                     "valu_issue_frac": valu / VALU_ISSUE_PEAK,
                     "per_launch": "8 flop x 1024 taps x 1000 tones x %.1f outputs" % (outs / launches)},
        "config": {"workload": w.name + ", 2^27 int16 I/Q samples in 2^23-sample buffers",
                   "ntones": int(w.words.size), "T": int(w.h.size), "D": w.D,
                   "buffer_samples": w.buffer},
    }, (w, d)


# ------------------------------------------------------------- large N

def bench_pcie(rf, torch, siggen, steps):
    """The production PFB stream fed from pinned host memory: each 2^24-sample
    buffer is copied over PCIe on a copy stream into one of two device staging
    buffers while the PFB of the previous buffer runs; spectra stay on the
    device.  The paper's own bottleneck was this host hop; reported beside the
    device-resident rate, never as `value`."""
    w = siggen.pfb_production()
    d = siggen.iq_torch(w.stream, 0, w.nsamples)
    host = torch.empty(d.numel(), dtype=torch.int16, pin_memory=True)
    host.copy_(d)
    del d
    nbuf = w.nsamples // w.buffer
    fpb = w.buffer // w.N
    stage = [torch.empty(2 * w.buffer, dtype=torch.int16, device="cuda") for _ in range(2)]
    out = torch.empty((nbuf, fpb, w.N), dtype=torch.complex64, device="cuda")
    p = rf.Pfb(w.N, w.M, w.h, max_samples_per_call=w.buffer)
    p.tune(w.buffer)
    comp = torch.cuda.current_stream()
    cs = torch.cuda.Stream()
    ready = [torch.cuda.Event() for _ in range(2)]
    done = [torch.cuda.Event() for _ in range(2)]

    def step():
        for b in range(nbuf):
            k = b & 1
            with torch.cuda.stream(cs):
                cs.wait_event(done[k])
                stage[k].copy_(host[2 * b * w.buffer: 2 * (b + 1) * w.buffer], non_blocking=True)
                ready[k].record(cs)
            comp.wait_event(ready[k])
            p.process_ptr(stage[k].data_ptr(), w.buffer, out.data_ptr() + 8 * b * fpb * w.N, fpb,
                          comp.cuda_stream)
            done[k].record(comp)

    for k in range(2):
        done[k].record(comp)
    step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(comp)
    cs.wait_event(e0)
    for _ in range(steps):
        step()
    e1.record(comp)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    p.close()
    samples = steps * w.nsamples
    return {"value": samples / sec / 1e6, "unit": "Msamples/s",
            "h2d_gbs": 4.0 * samples / sec / 1e9,
            "workload": "the N=1024 M=8 production stream from pinned host memory (2^24-sample "
                        "buffers over PCIe, copies overlapped with the PFB), spectra on the device"}


def bench_large(rf, torch, siggen, steps, warmup):
    """N = 10^5 channels (Sec. III.A, Fig. 3), M = 8, Kaiser(9): 2^27 samples of
    the production stream in 2^24-sample buffers, through the fold pass and
    the four-step FFT (N = 200 x 500)."""
    w = siggen.pfb_production()
    N, M = 100000, 8
    h = siggen.pfb_prototype(N, M, "kaiser", 9.0)
    nsamp = 1 << 27
    buf = 1 << 24
    d = siggen.iq_torch(w.stream, 0, nsamp)
    nbuf = nsamp // buf
    p = rf.Pfb(N, M, h, max_samples_per_call=buf)
    fmax = buf // N + 2
    out = torch.empty((nbuf, fmax, N), dtype=torch.complex64, device="cuda")
    s = torch.cuda.current_stream()
    sh = s.cuda_stream

    def step():
        for b in range(nbuf):
            p.process_ptr(d.data_ptr() + 4 * b * buf, buf, out.data_ptr() + 8 * b * fmax * N, fmax, sh)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        step()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kern_s = ms / 1e3 / (steps * nbuf)
    p.close()
    # device traffic of the three passes: fold 4 B in + 8 B out, two FFT
    # steps 16 B each per sample (12 B/sample is the method's minimum)
    return {"value": steps * nsamp / (ms / 1e3) / 1e6, "unit": "Msamples/s",
            "us_per_buffer": kern_s * 1e6,
            "hbm_gbs_44B_per_sample": 44.0 * buf / kern_s / 1e9,
            "config": {"workload": "pfb N=100000 M=8 kaiser9, 2^27 samples in 2^24-sample buffers, "
                                   "fold + four-step FFT (200 x 500)", "N": N, "M": M}}


# -------------------------------------------------------------------- Tx

def bench_tx(rf, torch, siggen, steps, warmup):
    """1000-tone transmit synthesis (the DDC bank's tones, 8 LSB each), 2^27
    samples per step in 16 buffers of 2^23; fixed and chirped tones."""
    w = siggen.ddc_bank()
    nbuf = w.nsamples // w.buffer
    amp = np.full(w.words.size, 8.0, dtype=np.float32)
    out = torch.empty(2 * w.buffer * nbuf, dtype=torch.int16, device="cuda")
    s = torch.cuda.current_stream()
    sh = s.cuda_stream
    res = {"config": {"workload": "tx 1000 tones, 2^27 int16 I/Q samples in 2^23-sample buffers",
                      "ntones": int(w.words.size), "buffer_samples": w.buffer}}
    crng = np.random.default_rng(34)
    cw = [siggen.chirp_words(float(crng.uniform(-90e6, 90e6)), float(crng.uniform(-2e13, 2e13)))
          for _ in range(w.words.size)]
    for name, inc, K in (("fixed", w.words, None),
                         ("chirped", np.array([a for a, _ in cw], np.uint64), np.array([b for _, b in cw], np.uint64))):
        tx = rf.Tx(inc, amp, w.phase0, K, max_samples_per_call=w.buffer)

        def step():
            for b in range(nbuf):
                tx.synthesize_ptr(out.data_ptr() + 4 * b * w.buffer, w.buffer, sh)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            step()
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        kern_s = ms / 1e3 / (steps * nbuf)
        # VALU issue: 12.25 (fixed) / 13.7 (chirped) instructions per sample-tone
        per = 12.25 if K is None else 13.7
        valu = per * w.words.size * w.buffer / kern_s
        res[name] = {"value": steps * w.nsamples / (ms / 1e3) / 1e6, "unit": "Msamples/s",
                     "kernel_us": kern_s * 1e6, "valu_issue_frac": valu / VALU_ISSUE_PEAK}
        log("tx %s: %.0f Msamples/s, %.1f us/launch" % (name, res[name]["value"], kern_s * 1e6))
        tx.close()
    return res, (w, amp)


def cpu_tx(oracle, w, amp, budget_s):
    """The oracle's Tx on the first k samples of the 1000-tone buffer, sized to ~budget_s."""
    def run(k):
        t0 = time.perf_counter()
        oracle.tx(w.phase0, w.words, amp, k)
        return time.perf_counter() - t0
    k = 4096
    t = run(k)
    for _ in range(2):     # the first probe is dominated by overheads: refine twice
        k = int(max(k, k * budget_s / max(t, 1e-6)))
        t = run(k)
    return {"value": k / t / 1e6, "unit": "Msamples/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "seconds": t, "sample": "first %d samples of the 1000-tone buffer, FP32 as the kernel, "
                                    "OpenMP over samples" % k}


# ------------------------------------------------------------- precision

MFMA_PEAK_TF = 2500.0          # MI355X dense FP16/BF16 MFMA, published


def bench_precision(rf, torch, siggen, oracle, steps, warmup):
    """N=256, M=8, Kaiser(9), 2^22 frames: FP32 FFT vs DFT on FP16 / BF16 MFMA (hi/lo)."""
    w = siggen.pfb_precision()
    nf = 1 << 22
    log("precision: generating %d samples on the device" % w.nsamples)
    d = siggen.iq_torch(w.stream, 0, w.nsamples)
    out = torch.empty((nf, w.N), dtype=torch.complex64, device="cuda")
    s = torch.cuda.current_stream()
    sh = s.cuda_stream
    # reference frames: 8 blocks of 128 frames spread over the stream
    rng = np.random.default_rng(4)
    starts = sorted(rng.choice(nf // 128, size=8, replace=False) * 128)
    refs = []
    span = w.N * w.M
    for f0 in starts:
        iq = d[2 * f0 * w.N: 2 * ((f0 + 127) * w.N + span)].cpu().numpy()
        refs.append(oracle.pfb(np.asarray(w.h, np.float32).astype(np.float64), w.N, w.M, iq=iq))
    res = {"config": {"workload": w.name, "N": w.N, "M": w.M, "frames": nf,
                      "samples": w.nsamples}}
    for name, mode in (("fft_f32", 0), ("mfma_f16x2", 1), ("mfma_bf16x2", 2)):
        p = rf.Pfb(w.N, w.M, w.h, dft_mode=mode, max_samples_per_call=w.nsamples)

        def once():
            p.reset()
            got = p.process_ptr(d.data_ptr(), w.nsamples, out.data_ptr(), nf, sh)
            assert got == nf

        for _ in range(warmup):
            once()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tot = 0.0
        for _ in range(steps):
            p.reset()
            e0.record(s)
            p.process_ptr(d.data_ptr(), w.nsamples, out.data_ptr(), nf, sh)
            e1.record(s)
            torch.cuda.synchronize()
            tot += e0.elapsed_time(e1)
        ms = tot / steps
        once()
        torch.cuda.synchronize()
        snr = []
        for f0, ref in zip(starts, refs):
            y = out[f0: f0 + 128].cpu().numpy().astype(np.complex128)
            snr.append((np.sum(np.abs(ref) ** 2, 0), np.sum(np.abs(y - ref) ** 2, 0)))
        num = sum(a for a, _ in snr)
        den = sum(b for _, b in snr)
        ch = 10 * np.log10(num / np.maximum(den, 1e-300))
        r = {"ms": ms, "msamples_per_s": w.nsamples / (ms / 1e3) / 1e6,
             "hbm_frac": 12.0 * w.nsamples / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
             "channel_snr_db": {"min": float(ch.min()), "median": float(np.median(ch)),
                                "max": float(ch.max())}}
        if mode:
            flop = 2.0 * 2 * 3 * 32 * 32 * 16 * nf    # 2 GEMM stages x 3 hi/lo terms per frame
            r["mfma_tflops"] = flop / (ms / 1e3) / 1e12
            r["mfma_frac"] = r["mfma_tflops"] / MFMA_PEAK_TF
            prof = profiled_mfma()
            if prof:
                for kname, kr in prof.items():
                    if ("RF_PREC_BF16" in kname or ", 2>" in kname) == (mode == 2):
                        r["mfma_busy_counter"] = {"kernel": kname, "busy_frac": kr["mfma_busy_frac"],
                                                  "source": os.path.relpath(MFMA_PROFILE, ROOT)}
        res[name] = r
        log("precision %s: %.3f ms, SNR min %.1f dB" % (name, ms, ch.min()))
        p.close()
    return res


# --------------------------------------------------------------- serving

def bench_serving(rf, torch, seconds):
    """16-stream mix (Poisson arrivals, 1.6 Gs/s offered): latency and throughput per mode."""
    from paper_1812_02200_amd import serve
    from siggen import mix
    specs, arrivals = mix.build_mix(duration_s=seconds)
    log("serving: %d streams, %d buffers over %.1f s" % (len(specs), len(arrivals), seconds))
    pool = mix.make_pool()
    torch.cuda.synchronize()
    res = {"config": {"workload": "16 streams, N in {64,256,1024,4096}, M in {4,8}, 8 with DDC "
                                  "banks of 10-2000 tones (T=1024, D=1000), buffers 2^16..2^24, "
                                  "Poisson arrivals at 1.6 Gs/s", "seconds": seconds,
                      "buffers": len(arrivals)}}
    modes = (("graph", rf.RFS_MODE_GRAPH), ("batched", rf.RFS_MODE_BATCHED),
             ("sequential", rf.RFS_MODE_SEQUENTIAL))
    for name, m in modes:
        r = serve.run(specs, arrivals, pool, m, realtime=True)
        res[name] = {"latency_ms": r["latency_ms"], "msamples_per_s": r["msamples_per_s"],
                     "batches": r["batches"]}
        log("serving %s: p50 %.2f ms p99 %.2f ms" % (name, r["latency_ms"]["p50"], r["latency_ms"]["p99"]))
    for name, m in modes:
        r = serve.run(specs, arrivals, pool, m, realtime=False)
        res[name]["saturation_msamples_per_s"] = r["msamples_per_s"]
        log("serving %s saturation: %.0f Msamples/s" % (name, r["msamples_per_s"]))
    # the same arrivals from pinned host memory: each buffer is copied to a
    # device staging slot by the server's copy stream (PCIe inside the latency)
    host_pool = torch.empty(pool.shape, dtype=pool.dtype, pin_memory=True)
    host_pool.copy_(pool)
    torch.cuda.synchronize()
    for name, m in (("graph", rf.RFS_MODE_GRAPH), ("sequential", rf.RFS_MODE_SEQUENTIAL)):
        r = serve.run(specs, arrivals, host_pool, m, realtime=True, host_slots=2)
        res[name + "_host_arrivals"] = {"latency_ms": r["latency_ms"], "msamples_per_s": r["msamples_per_s"],
                                        "batches": r["batches"]}
        log("serving %s, host arrivals: p50 %.2f ms p99 %.2f ms"
            % (name, r["latency_ms"]["p50"], r["latency_ms"]["p99"]))
    del host_pool
    return res


def cpu_ddc(oracle, w, d, budget_s):
    """The FP64 oracle on the first outputs of every tone, sized to ~budget_s of CPU work."""
    iq = d.cpu().numpy()
    nout = oracle.ddc_noutputs(w.nsamples, w.h.size, w.D)
    ntones = w.words.size

    def run(k):
        ti = np.repeat(np.arange(ntones), k)
        oi = np.tile(np.arange(k), ntones)
        t0 = time.perf_counter()
        oracle.ddc_points(w.words, w.phase0, w.h, w.D, ti, oi, iq=iq)
        return time.perf_counter() - t0

    k = 8
    t = run(k)
    k = int(min(nout, max(k, k * budget_s / max(t, 1e-6))))
    t = run(k)
    # k outputs of every tone cover k*D input samples of the 1000-tone bank
    return {"value": k * w.D / t / 1e6, "unit": "Msamples/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": t, "cpu_model": cpu_model(),
            "sample": "first %d outputs of all %d tones (%d input samples), FP64, OpenMP over points"
                      % (k, ntones, k * w.D)}


def main():
    a = parse()
    if a.pmc_summary:
        pmc_summary(*a.pmc_summary)
        return
    if a.trace_summary:
        trace_summary(a.trace_summary, a.bench_out)
        return
    if a.mfma_summary:
        mfma_summary(a.mfma_summary)
        return
    if a.pfb_shape:
        SHAPES["pfb"] = a.pfb_shape
    if a.ddc_grid:
        SHAPES["ddc"] = a.ddc_grid
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus %d is not supported" % a.gpus}))
        sys.exit(2)
    import torch
    import siggen
    import paper_1812_02200_amd as rf
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU available"}))
        sys.exit(1)
    torch.cuda.set_device(0)
    rec = {"metric": METRIC, "value": None, "unit": "Msamples/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {}, "device": torch.cuda.get_device_name(0)}
    keep = {}
    legs = set(a.workload.split(","))
    bad = legs - {"all", "pfb", "ddc", "tx", "large", "precision", "serving", "copyprobe"}
    if bad or ("copyprobe" in legs and len(legs) > 1):
        print(json.dumps({"error": "unknown or mixed workloads: %s" % a.workload}))
        sys.exit(2)

    def want(leg):
        return "all" in legs or leg in legs

    if legs == {"copyprobe"}:
        print(json.dumps(bench_copyprobe(torch)))
        return
    if want("pfb"):
        r, keep["pfb"] = bench_pfb(rf, torch, siggen, a.steps, a.warmup)
        rec["value"] = r["value"]
        rec["ms_per_step"] = r["ms_per_step"]
        rec["config"] = r.pop("config")
        rec["roofline"] = r.pop("roofline")
        rec["pfb"] = r
        log("pfb: %.0f Msamples/s, %.1f us/launch" % (r["value"], r["kernel_us"]))
        if not SHAPES.get("pfb"):   # (a pinned shape means a profiling run of the timed kernel)
            rec["pfb"]["pcie_inclusive"] = bench_pcie(rf, torch, siggen, max(1, min(a.steps, 3)))
            log("pfb from pinned host memory: %.0f Msamples/s (%.1f GB/s over PCIe)" %
                (rec["pfb"]["pcie_inclusive"]["value"], rec["pfb"]["pcie_inclusive"]["h2d_gbs"]))
    if want("ddc"):
        r, keep["ddc"] = bench_ddc(rf, torch, siggen, a.steps, a.warmup)
        rec["ddc"] = r
        if rec["value"] is None:
            rec["value"] = r["value"]
            rec["ms_per_step"] = r["ms_per_step"]
            rec["config"] = r["config"]
            rec["roofline"] = r["roofline"]
        log("ddc: %.0f Msamples/s, %.1f us/launch" % (r["value"], r["kernel_us"]))
    if want("large"):
        rec["large_n"] = bench_large(rf, torch, siggen, max(1, min(a.steps, 5)), 1)
        log("large N=10^5: %.0f Msamples/s" % rec["large_n"]["value"])
        if rec["value"] is None:
            rec["value"] = rec["large_n"]["value"]
            rec["config"] = rec["large_n"]["config"]
    if want("tx"):
        r, keep["tx"] = bench_tx(rf, torch, siggen, a.steps, a.warmup)
        rec["tx"] = r
        if rec["value"] is None:
            rec["value"] = r["fixed"]["value"]
            rec["config"] = r["config"]
    if want("precision"):
        import oracle
        rec["precision"] = bench_precision(rf, torch, siggen, oracle, max(1, min(a.steps, 5)), 1)
    if want("serving"):
        rec["serving"] = bench_serving(rf, torch, a.serve_seconds)
        rec["p99_buffer_latency_ms"] = rec["serving"]["graph"]["latency_ms"]["p99"]
    if not a.no_cpu_baseline:
        import oracle
        if "pfb" in keep:
            rec["cpu_baseline"] = cpu_pfb(oracle, *keep["pfb"], a.cpu_seconds)
        if "ddc" in keep:
            cb = cpu_ddc(oracle, *keep["ddc"], a.cpu_seconds)
            if "cpu_baseline" in rec:
                rec["ddc"]["cpu_baseline"] = cb
            else:
                rec["cpu_baseline"] = cb
        if "tx" in keep:
            cb = cpu_tx(oracle, *keep["tx"], a.cpu_seconds / 2)
            if "cpu_baseline" in rec:
                rec["tx"]["cpu_baseline"] = cb
            else:
                rec["cpu_baseline"] = cb
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
