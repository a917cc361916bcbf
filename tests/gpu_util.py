"""Helpers shared by the GPU tests: device handles, error metrics, buffer splitting."""
from __future__ import annotations

import sys

import numpy as np

FS = 8192.0   # 14-bit full scale in LSB


def need_gpu():
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(iq_np):
    import torch
    return torch.from_numpy(np.ascontiguousarray(iq_np, dtype=np.int16)).cuda()


def f32(h):
    """Taps as the GPU sees them (FP32), promoted back to FP64 for the oracle."""
    return np.asarray(h, dtype=np.float32).astype(np.float64)


def err_fs(y, ref, dc_gain):
    """RMS error in units of a full-scale tone's output: ||e|| / (sqrt(count) * 8192 * sum h)."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    assert y.shape == ref.shape, (y.shape, ref.shape)
    if ref.size == 0:
        return 0.0
    return float(np.linalg.norm(y - ref) / (np.sqrt(ref.size) * FS * abs(dc_gain)))


def err_rel(y, ref):
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(y - ref) / nr) if nr > 0 else float(np.linalg.norm(y))


U32 = 2.0 ** -24   # FP32 unit roundoff


def iq_abs(iq):
    """|x| of interleaved int16 I/Q samples (float64)."""
    a = np.asarray(iq, dtype=np.float64).reshape(-1, 2)
    return np.hypot(a[:, 0], a[:, 1])


def pfb_abs_mass(h, N, M, iq, frames):
    """A_p = sum_i |h[i]| |x[pN + i]| over frame p's N*M products (the oracle's
    frame p covers samples pN .. pN + NM - 1 with weight h[i])."""
    ah = np.abs(np.asarray(h, dtype=np.float64))
    return np.array([float(ah @ iq_abs(iq[2 * p * N: 2 * (p * N + N * M)])) for p in frames])


def check_pfb_elements(y, ref, h, N, M, iq, frames=None):
    """Element-wise bar for an FP32 PFB frame: every bin's error is at most
    c u A_p with c = 2 (M + 8 log2 N + 16).  The fold's M-term sums of FP32
    products err by at most (M + 1) u times their |h||x| mass; each FFT stage
    adds at most (log2 r + 4) u sqrt(2) times the sum of |v| (the butterfly's
    adds, the twiddle product and the twiddle's own rounding), and every
    intermediate value is bounded by sum |v| <= A_p; the factor 2 is margin.
    A single wrong bin exceeds it by orders of magnitude (a bin of a noise frame
    is about A_p / sqrt(N M)).  Returns the largest |e| / bound."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    if ref.size == 0:
        return 0.0
    if frames is None:
        frames = range(ref.shape[0])
    A = pfb_abs_mass(h, N, M, iq, frames)
    bound = 2.0 * (M + 8.0 * np.log2(N) + 16.0) * U32 * A
    emax = np.abs(y - ref).max(axis=1)
    ratio = float(np.max(emax / np.maximum(bound, 1e-300)))
    log("  max|e| per frame / FP32 bound = %.3g (max|e| = %.3g LSB)" % (ratio, float(emax.max())))
    assert np.all(emax <= bound), ratio
    return ratio


def check_ddc_elements(y, ref, h, D, iq, tones=None, outs=None):
    """Element-wise bar for FP32 DDC outputs: |e| <= 2 (T + 8) u B_n with
    B_n = sum_j |h[T-1-j]| |x[nD + j]|.  Each output component is a chain of
    T/2 FMAs per partial sum (four partials, two terms per sample) plus two
    adds; the terms' magnitudes sum to at most sqrt(2) B_n, and the product
    h x and the FP32 table entries add one rounding each; the factor 2 is
    margin.  Row-major y/ref [tones x outputs], or 1-D samples at (tones, outs).
    Returns the largest |e| / bound."""
    y = np.asarray(y, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    if ref.size == 0:
        return 0.0
    ah = np.abs(np.asarray(h, dtype=np.float64))[::-1]
    T = ah.size
    if outs is None:
        outs = np.arange(ref.shape[1])
    B = np.array([float(ah @ iq_abs(iq[2 * o * D: 2 * (o * D + T)])) for o in np.asarray(outs)])
    bound = 2.0 * (T + 8.0) * U32 * B
    e = np.abs(y - ref)
    if tones is None:
        bound = bound[None, :]
    ratio = float(np.max(e / np.maximum(bound, 1e-300)))
    log("  max|e| / FP32 bound = %.3g (max|e| = %.3g)" % (ratio, float(e.max())))
    assert np.all(e <= bound), ratio
    return ratio


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_pfb(pfb, iq_dev, sizes, torch):
    """Feed iq_dev (int16 interleaved) in buffers of the given sizes; return all frames (numpy)."""
    outs = []
    pos = 0
    for n in sizes:
        F = pfb.frames_for(n)
        out = torch.empty((max(F, 1), pfb.width), dtype=torch.complex64, device="cuda")
        y = pfb.process(iq_dev[2 * pos: 2 * (pos + n)], out=out)
        assert y.shape[0] == F
        outs.append(y)
        pos += n
    torch.cuda.synchronize()
    return torch.cat(outs, 0).cpu().numpy() if outs else np.zeros((0, pfb.width), np.complex64)


def run_ddc(ddc, iq_dev, sizes, torch):
    outs = []
    pos = 0
    for n in sizes:
        no = ddc.outputs_for(n)
        out = torch.empty((ddc.ntones, max(no, 1)), dtype=torch.complex64, device="cuda")
        y = ddc.process(iq_dev[2 * pos: 2 * (pos + n)], out=out)
        assert y.shape[1] == no
        outs.append(y)
        pos += n
    torch.cuda.synchronize()
    return torch.cat(outs, 1).cpu().numpy()
