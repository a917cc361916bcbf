"""ctypes binding of librfchan.so (the C ABI declared in include/rfchan.h).

Argument marshalling only: torch tensors supply device pointers and HIP stream
handles, every step of the computation runs in the library's HIP kernels.
There is no fallback: if the library is missing or a call fails, an exception
is raised.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librfchan.so")

RF_OK = 0
RF_EINVAL = 1
RF_ENOMEM = 2
RF_EDEVICE = 3
RF_ECAPACITY = 4
RF_EAGAIN = 5
RF_EUNSUPPORTED = 6

RF_DFT_FFT_F32 = 0
RF_DFT_MFMA_F16X2 = 1
RF_DFT_MFMA_BF16X2 = 2

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t

RFS_PFB = 1
RFS_DDC = 2
RFS_MODE_SEQUENTIAL = 0
RFS_MODE_BATCHED = 1
RFS_MODE_GRAPH = 2


class StreamDesc(ctypes.Structure):
    _fields_ = [("kinds", ctypes.c_int32), ("nchan", ctypes.c_int32), ("ntaps", ctypes.c_int32),
                ("proto", ctypes.c_void_p), ("ntones", ctypes.c_int32),
                ("phase_inc", ctypes.c_void_p), ("phase0", ctypes.c_void_p),
                ("lpf_taps", ctypes.c_int32), ("lpf", ctypes.c_void_p), ("decim", ctypes.c_int32),
                ("max_buffer", ctypes.c_uint64), ("out_slots", ctypes.c_int32),
                ("host_slots", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_int32), ("slot", ctypes.c_int32), ("tag", ctypes.c_uint64),
                ("nsamples", ctypes.c_uint64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("pfb_frames", ctypes.c_uint64), ("pfb_out", ctypes.c_void_p),
                ("ddc_outputs", ctypes.c_uint64), ("ddc_ld", ctypes.c_uint64),
                ("ddc_out", ctypes.c_void_p), ("t_submit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("samples", ctypes.c_uint64), ("bytes_admitted", ctypes.c_uint64),
                ("bytes_budget", ctypes.c_uint64), ("streams_open", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("gpu_busy_seconds", ctypes.c_double)]


# name -> (restype, argtypes); mirrors include/rfchan.h
SIGNATURES = {
    "rf_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "rf_last_error": (ctypes.c_char_p, []),
    "rf_version": (ctypes.c_int, []),
    "pfb_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _I32, _P, _I32, _U64]),
    "pfb_frames_for": (_U64, [_P, _U64]),
    "pfb_process": (ctypes.c_int, [_P, _P, _U64, _P, _U64, ctypes.POINTER(_U64), _P]),
    "pfb_process_static": (ctypes.c_int, [_P, _P, _U64, _P, _U64, ctypes.POINTER(_U64), _P]),
    "pfb_counters": (ctypes.c_int, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "pfb_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(_SZ)]),
    "pfb_set_state": (ctypes.c_int, [_P, _P, _SZ]),
    "pfb_reset": (ctypes.c_int, [_P]),
    "pfb_destroy": (ctypes.c_int, [_P]),
    "ddc_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _P, _P, _I32, _P, _I32, _U64]),
    "ddc_create_chirp": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _P, _P, _P, _I32, _P, _I32, _U64]),
    "pfb_set_channels": (ctypes.c_int, [_P, _P, _I32]),
    "tx_create": (ctypes.c_int, [ctypes.POINTER(_P), _I32, _P, _P, _P, _P, _U64]),
    "tx_synthesize": (ctypes.c_int, [_P, _P, _U64, _P]),
    "tx_set_tones": (ctypes.c_int, [_P, _P, _P, _P]),
    "tx_get_state": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(_U64)]),
    "tx_reset": (ctypes.c_int, [_P]),
    "tx_destroy": (ctypes.c_int, [_P]),
    "ddc_outputs_for": (_U64, [_P, _U64]),
    "ddc_process": (ctypes.c_int, [_P, _P, _U64, _P, _U64, ctypes.POINTER(_U64), _P]),
    "ddc_get_phase": (ctypes.c_int, [_P, _P]),
    "ddc_counters": (ctypes.c_int, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_U64), ctypes.POINTER(_U64)]),
    "ddc_get_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(_SZ)]),
    "ddc_set_state": (ctypes.c_int, [_P, _P, _SZ]),
    "ddc_reset": (ctypes.c_int, [_P]),
    "ddc_destroy": (ctypes.c_int, [_P]),
    "pfb_tune": (ctypes.c_int, [_P, _U64, _P, ctypes.POINTER(ctypes.c_double)]),
    "pfb_apply_tuned": (ctypes.c_int, [_P, _U64]),
    "pfb_tuned_config": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "ddc_tune": (ctypes.c_int, [_P, _U64, _P, ctypes.POINTER(ctypes.c_double)]),
    "ddc_apply_tuned": (ctypes.c_int, [_P, _U64]),
    "ddc_tuned_config": (ctypes.c_int, [_P, ctypes.POINTER(_I32)]),
    "rfs_create": (ctypes.c_int, [ctypes.POINTER(_P), _U64, _I32, _I32]),
    "rfs_stream_footprint": (_U64, [ctypes.POINTER(StreamDesc)]),
    "rfs_open_stream": (ctypes.c_int, [_P, ctypes.POINTER(StreamDesc), ctypes.POINTER(_I32)]),
    "rfs_submit": (ctypes.c_int, [_P, _I32, _P, _U64, _U64]),
    "rfs_poll": (ctypes.c_int, [_P, ctypes.POINTER(Completion), _I32, ctypes.POINTER(_I32), _I32]),
    "rfs_release": (ctypes.c_int, [_P, _I32, _I32]),
    "rfs_close_stream": (ctypes.c_int, [_P, _I32]),
    "rfs_get_stats": (ctypes.c_int, [_P, ctypes.POINTER(Stats)]),
    "rfs_now": (ctypes.c_double, []),
    "rfs_destroy": (ctypes.c_int, [_P]),
}

_lock = threading.Lock()
_lib = None


class RfError(RuntimeError):
    def __init__(self, status: int, call: str, detail: str):
        super().__init__("%s failed: %s (%s)" % (call, detail or "", status_name(status)))
        self.status = status


def status_name(status: int) -> str:
    return {0: "RF_OK", 1: "RF_EINVAL", 2: "RF_ENOMEM", 3: "RF_EDEVICE", 4: "RF_ECAPACITY",
            5: "RF_EAGAIN", 6: "RF_EUNSUPPORTED"}.get(status, "status %d" % status)


def lib():
    """Load librfchan.so once (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "librfchan.so is not built (%s); run `python -m paper_1812_02200_amd.build`"
                    % LIB_PATH)
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
        return _lib


def check(status: int, call: str) -> None:
    if status != RF_OK:
        detail = lib().rf_last_error().decode(errors="replace")
        raise RfError(status, call, detail)


def version() -> int:
    return int(lib().rf_version())


def _torch():
    import torch  # noqa: WPS433 (device memory and streams only)
    return torch


def _stream_handle(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _check_iq(iq):
    torch = _torch()
    if not isinstance(iq, torch.Tensor) or iq.dtype != torch.int16 or not iq.is_cuda:
        raise TypeError("iq must be an int16 CUDA/HIP tensor of interleaved I/Q")
    if not iq.is_contiguous():
        raise ValueError("iq must be contiguous")
    if iq.numel() % 2:
        raise ValueError("iq must hold an even number of int16 (I/Q pairs)")
    return iq.numel() // 2


class Pfb:
    """Polyphase filter-bank channelizer handle (pfb_* calls)."""

    def __init__(self, nchan: int, ntaps: int, proto, dft_mode: int = RF_DFT_FFT_F32,
                 max_samples_per_call: int = 1 << 24):
        import numpy as np
        h = np.ascontiguousarray(np.asarray(proto, dtype=np.float32).reshape(-1))
        if h.size != nchan * ntaps:
            raise ValueError("prototype needs nchan*ntaps = %d taps" % (nchan * ntaps))
        self.N, self.M = int(nchan), int(ntaps)
        self._h = _P()
        check(lib().pfb_create(ctypes.byref(self._h), self.N, self.M, h.ctypes.data, int(dft_mode),
                               int(max_samples_per_call)), "pfb_create")
        self.max_samples = int(max_samples_per_call)
        self.width = self.N            # values per output frame (N, or the chosen channels)

    def frames_for(self, nsamples: int) -> int:
        return int(lib().pfb_frames_for(self._h, int(nsamples)))

    def set_channels(self, channels=None) -> None:
        """Return only these bins (in this order) from now on; None: all N bins."""
        import numpy as np
        if channels is None:
            check(lib().pfb_set_channels(self._h, None, 0), "pfb_set_channels")
            self.width = self.N
            return
        ch = np.ascontiguousarray(np.asarray(channels, dtype=np.int32).reshape(-1))
        check(lib().pfb_set_channels(self._h, ch.ctypes.data if ch.size else None, int(ch.size)),
              "pfb_set_channels")
        self.width = int(ch.size) if ch.size else self.N

    def process(self, iq, out=None, stream=None):
        """Channelize int16 I/Q tensor `iq`; returns a complex64 tensor [frames, width]."""
        torch = _torch()
        n = _check_iq(iq)
        F = self.frames_for(n)
        if out is None:
            out = torch.empty((max(F, 1), self.width), dtype=torch.complex64, device=iq.device)
        if out.dtype != torch.complex64 or not out.is_contiguous():
            raise TypeError("out must be a contiguous complex64 tensor")
        cap = out.numel() // self.width
        got = _U64(0)
        check(lib().pfb_process(self._h, iq.data_ptr() if n else None, n, out.data_ptr(), cap,
                                ctypes.byref(got), _stream_handle(stream)), "pfb_process")
        return out.view(-1, self.width)[: got.value]

    def process_ptr(self, iq_ptr: int, nsamples: int, out_ptr: int, out_cap_frames: int,
                    stream_handle: int) -> int:
        got = _U64(0)
        check(lib().pfb_process(self._h, iq_ptr, nsamples, out_ptr, out_cap_frames,
                                ctypes.byref(got), stream_handle), "pfb_process")
        return got.value

    def process_static_ptr(self, iq_ptr: int, nsamples: int, out_ptr: int, out_cap_frames: int,
                           stream_handle: int) -> int:
        """pfb_process_static: as process_ptr, scratch from the library's static array."""
        got = _U64(0)
        check(lib().pfb_process_static(self._h, iq_ptr, nsamples, out_ptr, out_cap_frames,
                                       ctypes.byref(got), stream_handle), "pfb_process_static")
        return got.value

    def tune(self, nsamples: int, stream=None):
        """Autotune the launch configuration for buffers of `nsamples`; returns
        (microseconds per launch, run_len, variant)."""
        us = ctypes.c_double(0)
        check(lib().pfb_tune(self._h, int(nsamples), _stream_handle(stream), ctypes.byref(us)), "pfb_tune")
        rl, var = self.tuned_config()
        return us.value, rl, var

    def tuned_config(self):
        """(run_len, variant) the next launches use (0: the built-in heuristic)."""
        rl, var = _I32(), _I32()
        check(lib().pfb_tuned_config(self._h, ctypes.byref(rl), ctypes.byref(var)), "pfb_tuned_config")
        return rl.value, var.value

    def apply_tuned(self, nsamples: int) -> bool:
        st = lib().pfb_apply_tuned(self._h, int(nsamples))
        if st == RF_EAGAIN:
            return False
        check(st, "pfb_apply_tuned")
        return True

    def counters(self):
        a, b, c = _U64(), _U64(), _U64()
        check(lib().pfb_counters(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "pfb_counters")
        return a.value, b.value, c.value

    def get_state(self) -> bytes:
        sz = _SZ(0)
        check(lib().pfb_get_state(self._h, None, ctypes.byref(sz)), "pfb_get_state")
        buf = ctypes.create_string_buffer(sz.value)
        check(lib().pfb_get_state(self._h, buf, ctypes.byref(sz)), "pfb_get_state")
        return buf.raw[: sz.value]

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().pfb_set_state(self._h, buf, len(blob)), "pfb_set_state")

    def reset(self) -> None:
        check(lib().pfb_reset(self._h), "pfb_reset")

    def close(self) -> None:
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            check(lib().pfb_destroy(h), "pfb_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ddc:
    """Direct-demodulation bank handle (ddc_* calls)."""

    def __init__(self, phase_inc, lpf, decim: int, phase0=None,
                 max_samples_per_call: int = 1 << 24, chirp=None):
        """chirp: per-tone phase second differences (ddc_create_chirp) for
        chirped tones, or None for ordinary tones (ddc_create)."""
        import numpy as np
        inc = np.ascontiguousarray(np.asarray(phase_inc, dtype=np.uint64).reshape(-1))
        p0 = None if phase0 is None else np.ascontiguousarray(
            np.asarray(phase0, dtype=np.uint64).reshape(-1))
        if p0 is not None and p0.size != inc.size:
            raise ValueError("phase0 must have one entry per tone")
        ck = None if chirp is None else np.ascontiguousarray(
            np.asarray(chirp, dtype=np.uint64).reshape(-1))
        if ck is not None and ck.size != inc.size:
            raise ValueError("chirp must have one entry per tone")
        h = np.ascontiguousarray(np.asarray(lpf, dtype=np.float32).reshape(-1))
        self.ntones, self.T, self.D = int(inc.size), int(h.size), int(decim)
        self._h = _P()
        p0p = None if p0 is None else p0.ctypes.data
        if ck is None:
            check(lib().ddc_create(ctypes.byref(self._h), self.ntones, inc.ctypes.data, p0p, self.T,
                                   h.ctypes.data, self.D, int(max_samples_per_call)), "ddc_create")
        else:
            check(lib().ddc_create_chirp(ctypes.byref(self._h), self.ntones, inc.ctypes.data, p0p,
                                         ck.ctypes.data, self.T, h.ctypes.data, self.D,
                                         int(max_samples_per_call)), "ddc_create_chirp")
        self.max_samples = int(max_samples_per_call)

    def outputs_for(self, nsamples: int) -> int:
        return int(lib().ddc_outputs_for(self._h, int(nsamples)))

    def process(self, iq, out=None, stream=None):
        """Demodulate int16 I/Q tensor `iq`; returns complex64 [ntones, nout] (a view of out)."""
        torch = _torch()
        n = _check_iq(iq)
        nout = self.outputs_for(n)
        if out is None:
            out = torch.empty((self.ntones, max(nout, 1)), dtype=torch.complex64, device=iq.device)
        if out.dtype != torch.complex64 or out.dim() != 2 or out.shape[0] != self.ntones:
            raise TypeError("out must be complex64 [ntones, ld]")
        if out.stride(1) != 1:
            raise ValueError("out rows must be contiguous")
        ld = out.stride(0)
        got = _U64(0)
        check(lib().ddc_process(self._h, iq.data_ptr() if n else None, n, out.data_ptr(), ld,
                                ctypes.byref(got), _stream_handle(stream)), "ddc_process")
        return out[:, : got.value]

    def process_ptr(self, iq_ptr: int, nsamples: int, out_ptr: int, ld: int,
                    stream_handle: int) -> int:
        got = _U64(0)
        check(lib().ddc_process(self._h, iq_ptr, nsamples, out_ptr, ld, ctypes.byref(got),
                                stream_handle), "ddc_process")
        return got.value

    def tune(self, nsamples: int, stream=None):
        """Autotune the persistent grid for buffers of `nsamples`; returns (us, grid)."""
        us = ctypes.c_double(0)
        check(lib().ddc_tune(self._h, int(nsamples), _stream_handle(stream), ctypes.byref(us)), "ddc_tune")
        return us.value, self.tuned_config()

    def tuned_config(self) -> int:
        """The persistent grid the next launches use (0: the built-in default)."""
        g = _I32()
        check(lib().ddc_tuned_config(self._h, ctypes.byref(g)), "ddc_tuned_config")
        return g.value

    def apply_tuned(self, nsamples: int) -> bool:
        st = lib().ddc_apply_tuned(self._h, int(nsamples))
        if st == RF_EAGAIN:
            return False
        check(st, "ddc_apply_tuned")
        return True

    def phase(self):
        import numpy as np
        out = np.empty(self.ntones, dtype=np.uint64)
        check(lib().ddc_get_phase(self._h, out.ctypes.data), "ddc_get_phase")
        return out

    def counters(self):
        a, b, c = _U64(), _U64(), _U64()
        check(lib().ddc_counters(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "ddc_counters")
        return a.value, b.value, c.value

    def get_state(self) -> bytes:
        sz = _SZ(0)
        check(lib().ddc_get_state(self._h, None, ctypes.byref(sz)), "ddc_get_state")
        buf = ctypes.create_string_buffer(sz.value)
        check(lib().ddc_get_state(self._h, buf, ctypes.byref(sz)), "ddc_get_state")
        return buf.raw[: sz.value]

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        check(lib().ddc_set_state(self._h, buf, len(blob)), "ddc_set_state")

    def reset(self) -> None:
        check(lib().ddc_reset(self._h), "ddc_reset")

    def close(self) -> None:
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            check(lib().ddc_destroy(h), "ddc_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tx:
    """Multi-tone transmit synthesis handle (tx_* calls): int16 I/Q DAC buffers."""

    def __init__(self, phase_inc, amplitude, phase0=None, chirp=None,
                 max_samples_per_call: int = 1 << 24):
        import numpy as np
        inc = np.ascontiguousarray(np.asarray(phase_inc, dtype=np.uint64).reshape(-1))
        amp = np.ascontiguousarray(np.asarray(amplitude, dtype=np.float32).reshape(-1))
        p0 = None if phase0 is None else np.ascontiguousarray(np.asarray(phase0, dtype=np.uint64).reshape(-1))
        ck = None if chirp is None else np.ascontiguousarray(np.asarray(chirp, dtype=np.uint64).reshape(-1))
        for name, arr in (("amplitude", amp), ("phase0", p0), ("chirp", ck)):
            if arr is not None and arr.size != inc.size:
                raise ValueError("%s must have one entry per tone" % name)
        self.ntones = int(inc.size)
        self.max_samples = int(max_samples_per_call)
        self._h = _P()
        check(lib().tx_create(ctypes.byref(self._h), self.ntones, inc.ctypes.data,
                              None if p0 is None else p0.ctypes.data,
                              None if ck is None else ck.ctypes.data, amp.ctypes.data,
                              self.max_samples), "tx_create")

    def synthesize(self, n: int, out=None, stream=None):
        """Next n samples as an int16 tensor [2n] (I/Q interleaved) on the current device."""
        torch = _torch()
        if out is None:
            out = torch.empty(2 * max(int(n), 1), dtype=torch.int16, device="cuda")
        if out.dtype != torch.int16 or not out.is_contiguous() or out.numel() < 2 * n:
            raise TypeError("out must be a contiguous int16 tensor of >= 2n elements")
        self.synthesize_ptr(out.data_ptr(), int(n), _stream_handle(stream))
        return out[: 2 * n]

    def synthesize_ptr(self, out_ptr: int, n: int, stream_handle) -> None:
        check(lib().tx_synthesize(self._h, out_ptr, int(n), stream_handle), "tx_synthesize")

    def set_tones(self, amplitude=None, phase_inc=None, chirp=None) -> None:
        import numpy as np
        arrs = []
        for arr, dt in ((amplitude, np.float32), (phase_inc, np.uint64), (chirp, np.uint64)):
            if arr is None:
                arrs.append(None)
                continue
            a = np.ascontiguousarray(np.asarray(arr, dtype=dt).reshape(-1))
            if a.size != self.ntones:
                raise ValueError("one entry per tone expected")
            arrs.append(a)
        check(lib().tx_set_tones(self._h, *[None if a is None else a.ctypes.data for a in arrs]),
              "tx_set_tones")

    def state(self):
        """(phase, rate, samples) at the next sample."""
        import numpy as np
        ph = np.empty(self.ntones, dtype=np.uint64)
        rt = np.empty(self.ntones, dtype=np.uint64)
        n = _U64(0)
        check(lib().tx_get_state(self._h, ph.ctypes.data, rt.ctypes.data, ctypes.byref(n)), "tx_get_state")
        return ph, rt, int(n.value)

    def reset(self) -> None:
        check(lib().tx_reset(self._h), "tx_reset")

    def close(self) -> None:
        if self._h:
            check(lib().tx_destroy(self._h), "tx_destroy")
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Multi-stream serving core (rfs_* calls): admission by device-memory
    footprint, continuous batching onto grouped kernels, optional hipGraph replay."""

    def __init__(self, hbm_budget_bytes: int, mode: int = RFS_MODE_GRAPH, max_streams: int = 64):
        self._h = _P()
        check(lib().rfs_create(ctypes.byref(self._h), int(hbm_budget_bytes), int(mode),
                               int(max_streams)), "rfs_create")
        self._keep = {}
        self._poll_buf = (Completion * 256)()

    @staticmethod
    def make_desc(pfb=None, ddc=None, max_buffer=1 << 20, out_slots=2, host_slots=0):
        """pfb=(N, M, proto); ddc=(words, phase0 or None, lpf, D); host_slots: device
        staging slots for pinned-host submissions.  Returns (desc, keepalive)."""
        import numpy as np
        d = StreamDesc()
        keep = []
        d.kinds = (RFS_PFB if pfb else 0) | (RFS_DDC if ddc else 0)
        if pfb:
            N, M, h = pfb
            h = np.ascontiguousarray(np.asarray(h, dtype=np.float32).reshape(-1))
            keep.append(h)
            d.nchan, d.ntaps, d.proto = int(N), int(M), h.ctypes.data
        if ddc:
            words, p0, lpf, D = ddc
            words = np.ascontiguousarray(np.asarray(words, dtype=np.uint64).reshape(-1))
            lpf = np.ascontiguousarray(np.asarray(lpf, dtype=np.float32).reshape(-1))
            keep += [words, lpf]
            d.ntones, d.phase_inc = int(words.size), words.ctypes.data
            if p0 is not None:
                p0 = np.ascontiguousarray(np.asarray(p0, dtype=np.uint64).reshape(-1))
                keep.append(p0)
                d.phase0 = p0.ctypes.data
            d.lpf_taps, d.lpf, d.decim = int(lpf.size), lpf.ctypes.data, int(D)
        d.max_buffer = int(max_buffer)
        d.out_slots = int(out_slots)
        d.host_slots = int(host_slots)
        return d, keep

    @staticmethod
    def footprint(desc) -> int:
        return int(lib().rfs_stream_footprint(ctypes.byref(desc)))

    def open_stream(self, desc, keep=None) -> int:
        sid = _I32(-1)
        check(lib().rfs_open_stream(self._h, ctypes.byref(desc), ctypes.byref(sid)), "rfs_open_stream")
        self._keep[sid.value] = keep
        return sid.value

    def try_open_stream(self, desc, keep=None):
        """Like open_stream, but returns None when the server answers RF_EAGAIN."""
        sid = _I32(-1)
        st = lib().rfs_open_stream(self._h, ctypes.byref(desc), ctypes.byref(sid))
        if st == RF_EAGAIN:
            return None
        check(st, "rfs_open_stream")
        self._keep[sid.value] = keep
        return sid.value

    def submit(self, sid: int, iq_ptr: int, nsamples: int, tag: int = 0) -> None:
        check(lib().rfs_submit(self._h, int(sid), iq_ptr, int(nsamples), int(tag)), "rfs_submit")

    def poll(self, max_n: int = 256, timeout_us: int = 0):
        n = _I32(0)
        max_n = min(max_n, len(self._poll_buf))
        check(lib().rfs_poll(self._h, self._poll_buf, max_n, ctypes.byref(n), int(timeout_us)), "rfs_poll")
        out = []
        for i in range(n.value):
            c = self._poll_buf[i]
            out.append({f: getattr(c, f) for f, _ in Completion._fields_ if f != "pad"})
        return out

    def release(self, sid: int, slot: int) -> None:
        check(lib().rfs_release(self._h, int(sid), int(slot)), "rfs_release")

    def close_stream(self, sid: int) -> None:
        check(lib().rfs_close_stream(self._h, int(sid)), "rfs_close_stream")
        self._keep.pop(sid, None)

    def stats(self) -> dict:
        st = Stats()
        check(lib().rfs_get_stats(self._h, ctypes.byref(st)), "rfs_get_stats")
        return {f: getattr(st, f) for f, _ in Stats._fields_ if f != "pad"}

    @staticmethod
    def now() -> float:
        return float(lib().rfs_now())

    def close(self) -> None:
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            check(lib().rfs_destroy(h), "rfs_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
