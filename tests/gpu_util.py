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
