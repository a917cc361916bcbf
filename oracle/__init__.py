"""FP64 CPU oracle for the PFB channelizer and the DDC bank (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``paper_1812_02200_amd``)
never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, double precision, OpenMP over
independent outputs); this module only builds it with gcc and marshals numpy
arrays through ctypes.  Definitions (paper Sec. III.A and III.B):

* PFB frame p (valid frames only, p*N + N*M <= S):
  ``X_p[k] = sum_n (sum_m h[mN+n] x[pN+mN+n]) exp(-2 pi i k n / N)``.
* DDC output n of tone t:
  ``y_t[n] = sum_k h[k] x[nD+T-1-k] conj(Tab[(phi0_t + m inc_t) >> 48])``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

GCC_FLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
             "-shared", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (in place)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int64
        U = ctypes.c_uint64
        lib.orc_dft_direct.argtypes = [P, I, P]
        lib.orc_fft_pow2.argtypes = [P, I]
        lib.orc_pfb_nframes.argtypes = [I, I, I]
        lib.orc_pfb_nframes.restype = I
        lib.orc_pfb_frames.argtypes = [P, P, I, I, I, P, P, I, P]
        lib.orc_pfb_fold_frames.argtypes = [P, P, I, I, I, P, P, I, P]
        lib.orc_nco_table.argtypes = [P]
        lib.orc_nco_phase.argtypes = [U, U, U]
        lib.orc_nco_phase.restype = U
        lib.orc_nco_phases.argtypes = [P, P, I, U, P]
        lib.orc_ddc_noutputs.argtypes = [I, I, I]
        lib.orc_ddc_noutputs.restype = I
        lib.orc_tab32.argtypes = [P]
        lib.orc_pfb_channels.argtypes = [P, P, I, I, I, P, P, I, P]
        lib.orc_tx.argtypes = [I, P, P, P, P, I, P]
        lib.orc_tx_advance.argtypes = [I, P, P, P, U]
        lib.orc_chirp_phase.argtypes = [U, U, U, U]
        lib.orc_chirp_phase.restype = U
        lib.orc_ddc.argtypes = [P, P, I, I, P, P, P, I, P, I, ctypes.c_int, P]
        lib.orc_ddc.restype = I
        lib.orc_ddc_points.argtypes = [P, P, I, P, P, P, I, P, I, P, P, I, ctypes.c_int, P]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = lib
        return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _stream_args(iq=None, x=None):
    """Return (iq int16 C-array or None, xc float64 C-array or None, S)."""
    if (iq is None) == (x is None):
        raise ValueError("pass exactly one of iq (int16 I/Q) or x (complex)")
    if iq is not None:
        iq = np.ascontiguousarray(iq, dtype=np.int16).reshape(-1)
        if iq.size % 2:
            raise ValueError("interleaved I/Q needs an even number of int16")
        return iq, None, iq.size // 2
    xc = np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).view(np.float64)
    return None, xc, xc.size // 2


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    _load().orc_set_num_threads(int(n))


def dft_direct(x) -> np.ndarray:
    """O(N^2) DFT by definition (complex128 in, complex128 out)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128))
    out = np.empty_like(x)
    _load().orc_dft_direct(_ptr(x.view(np.float64)), x.size, _ptr(out.view(np.float64)))
    return out


def fft_pow2(x) -> np.ndarray:
    """The oracle's own radix-2 FFT (N a power of two)."""
    x = np.array(x, dtype=np.complex128, copy=True)
    n = x.size
    if n & (n - 1):
        raise ValueError("N must be a power of two")
    _load().orc_fft_pow2(_ptr(x.view(np.float64)), n)
    return x


def pfb_nframes(S: int, N: int, M: int) -> int:
    return int(_load().orc_pfb_nframes(S, N, M))


def pfb(h, N: int, M: int, iq=None, x=None, frames=None) -> np.ndarray:
    """PFB output, complex128 [len(frames) x N] (all valid frames by default)."""
    iqa, xc, S = _stream_args(iq, x)
    h = np.ascontiguousarray(h, dtype=np.float64)
    if h.size != N * M:
        raise ValueError("prototype length must be N*M")
    if frames is None:
        nf = pfb_nframes(S, N, M)
        fr = None
    else:
        fr = np.ascontiguousarray(frames, dtype=np.int64)
        nf = fr.size
    out = np.empty((nf, N), dtype=np.complex128)
    _load().orc_pfb_frames(_ptr(iqa), _ptr(xc), S, N, M, _ptr(h), _ptr(fr), nf,
                           _ptr(out.view(np.float64)))
    return out


def pfb_channels(h, N: int, M: int, channels, iq=None, x=None) -> np.ndarray:
    """Selected channels of every valid frame, complex128 [frames x len(channels)],
    by a direct DFT sum at those bins."""
    iqa, xc, S = _stream_args(iq, x)
    h = np.ascontiguousarray(h, dtype=np.float64)
    if h.size != N * M:
        raise ValueError("prototype length must be N*M")
    ch = np.ascontiguousarray(channels, dtype=np.int64)
    if ch.size and (ch.min() < 0 or ch.max() >= N):
        raise ValueError("channel out of range")
    nf = pfb_nframes(S, N, M)
    out = np.empty((nf, ch.size), dtype=np.complex128)
    _load().orc_pfb_channels(_ptr(iqa), _ptr(xc), S, N, M, _ptr(h), _ptr(ch), ch.size,
                             _ptr(out.view(np.float64)))
    return out


def pfb_fold(h, N: int, M: int, iq=None, x=None, frames=None) -> np.ndarray:
    """The FIR/fold step alone, complex128 [frames x N]."""
    iqa, xc, S = _stream_args(iq, x)
    h = np.ascontiguousarray(h, dtype=np.float64)
    if frames is None:
        nf = pfb_nframes(S, N, M)
        fr = None
    else:
        fr = np.ascontiguousarray(frames, dtype=np.int64)
        nf = fr.size
    out = np.empty((nf, N), dtype=np.complex128)
    _load().orc_pfb_fold_frames(_ptr(iqa), _ptr(xc), S, N, M, _ptr(h), _ptr(fr), nf,
                                _ptr(out.view(np.float64)))
    return out


def pfb_fold_fft(h, N: int, M: int, iq=None, x=None, frames=None) -> np.ndarray:
    """Every bin of the given frames (all valid frames by default), complex128
    [frames x N]: the oracle's FP64 fold, then numpy's FP64 FFT as the DFT step
    (paper Sec. III.A: X_p[k] = sum_n v_p[n] exp(-2 pi i k n / N); a library
    FFT of any length, including the large and non-power-of-two N of Fig. 3,
    where the oracle's own direct DFT is O(N^2) per frame).  Pinned against
    the direct DFT at sampled bins and the radix-2 oracle path."""
    v = pfb_fold(h, N, M, iq=iq, x=x, frames=frames)
    return np.fft.fft(v, axis=1)


def nco_table() -> np.ndarray:
    """complex128[65536]: cos + i sin at 2 pi idx / 2^16 (FP64)."""
    tab = np.empty(65536, dtype=np.complex128)
    _load().orc_nco_table(_ptr(tab.view(np.float64)))
    return tab


def nco_phase(phi0: int, inc: int, m: int) -> int:
    return int(_load().orc_nco_phase(phi0 & (2**64 - 1), inc & (2**64 - 1), m & (2**64 - 1)))


def chirp_phase(phi0: int, inc: int, K: int, m: int) -> int:
    """phi0 + m*inc + K*m(m-1)/2 mod 2^64 (quadratic NCO of Eq. 1)."""
    M64 = 2**64 - 1
    return int(_load().orc_chirp_phase(phi0 & M64, inc & M64, K & M64, m & M64))


def nco_phases(inc, phi0, S: int) -> np.ndarray:
    inc = np.ascontiguousarray(inc, dtype=np.uint64)
    p0 = None if phi0 is None else np.ascontiguousarray(phi0, dtype=np.uint64)
    out = np.empty_like(inc)
    _load().orc_nco_phases(_ptr(p0), _ptr(inc), inc.size, S, _ptr(out))
    return out


def ddc_noutputs(S: int, T: int, D: int) -> int:
    return int(_load().orc_ddc_noutputs(S, T, D))


def _chirp_arg(chirp, n):
    if chirp is None:
        return None
    c = np.ascontiguousarray(chirp, dtype=np.uint64)
    if c.shape != (n,):
        raise ValueError("chirp must hold one word per tone")
    return c


def ddc(inc, phi0, h, D: int, iq=None, x=None, exact_nco: bool = False, chirp=None) -> np.ndarray:
    """All DDC outputs, complex128 [ntones x nout] (tone-major).  chirp: K per
    tone for quadratic-phase (chirped) tones, None for the linear NCO."""
    iqa, xc, S = _stream_args(iq, x)
    inc = np.ascontiguousarray(inc, dtype=np.uint64)
    p0 = None if phi0 is None else np.ascontiguousarray(phi0, dtype=np.uint64)
    ck = _chirp_arg(chirp, inc.size)
    h = np.ascontiguousarray(h, dtype=np.float64)
    T = h.size
    nout = ddc_noutputs(S, T, D)
    out = np.empty((inc.size, nout), dtype=np.complex128)
    _load().orc_ddc(_ptr(iqa), _ptr(xc), S, inc.size, _ptr(inc), _ptr(p0), _ptr(ck), T, _ptr(h),
                    D, int(bool(exact_nco)), _ptr(out.view(np.float64)))
    return out


def ddc_points(inc, phi0, h, D: int, tone_idx, out_idx, iq=None, x=None,
               exact_nco: bool = False, chirp=None) -> np.ndarray:
    """Selected DDC outputs y[tone_idx[i], out_idx[i]], complex128 [npts]."""
    iqa, xc, S = _stream_args(iq, x)
    inc = np.ascontiguousarray(inc, dtype=np.uint64)
    p0 = None if phi0 is None else np.ascontiguousarray(phi0, dtype=np.uint64)
    ck = _chirp_arg(chirp, inc.size)
    h = np.ascontiguousarray(h, dtype=np.float64)
    ti = np.ascontiguousarray(tone_idx, dtype=np.int64)
    oi = np.ascontiguousarray(out_idx, dtype=np.int64)
    if ti.shape != oi.shape:
        raise ValueError("tone_idx and out_idx must have the same shape")
    if ti.size and (ti.min() < 0 or ti.max() >= inc.size):
        raise ValueError("tone index out of range")
    out = np.empty(ti.size, dtype=np.complex128)
    _load().orc_ddc_points(_ptr(iqa), _ptr(xc), S, _ptr(inc), _ptr(p0), _ptr(ck), h.size, _ptr(h), D,
                           _ptr(ti), _ptr(oi), ti.size, int(bool(exact_nco)),
                           _ptr(out.view(np.float64)))
    return out


# ------------------------------------------------------------------ Tx

def tab32() -> np.ndarray:
    """The FP32 cos/sin table [2^16, 2] by its quarter-wave definition."""
    tab = np.empty((65536, 2), dtype=np.float32)
    _load().orc_tab32(_ptr(tab))
    return tab


def tx(phase, rate, amp, n: int, chirp=None) -> np.ndarray:
    """n samples of the multi-tone transmit buffer, int16 interleaved I/Q [2n],
    from the oscillator state (phase, rate, chirp) at its first sample."""
    ph = np.ascontiguousarray(phase, dtype=np.uint64)
    rt = np.ascontiguousarray(rate, dtype=np.uint64)
    a = np.ascontiguousarray(amp, dtype=np.float32)
    if rt.shape != ph.shape or a.shape != ph.shape:
        raise ValueError("phase, rate and amp need one entry per tone")
    ck = _chirp_arg(chirp, ph.size)
    out = np.empty(2 * n, dtype=np.int16)
    _load().orc_tx(ph.size, _ptr(ph), _ptr(rt), _ptr(ck), _ptr(a), n, _ptr(out))
    return out


def tx_advance(phase, rate, n: int, chirp=None):
    """Oscillator state (phase, rate) after n samples."""
    ph = np.array(phase, dtype=np.uint64)
    rt = np.array(rate, dtype=np.uint64)
    ck = _chirp_arg(chirp, ph.size)
    _load().orc_tx_advance(ph.size, _ptr(ph), _ptr(rt), _ptr(ck), n)
    return ph, rt
