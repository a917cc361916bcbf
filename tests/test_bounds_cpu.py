"""The element-wise FP32 error bars of the GPU parity tests, checked on the CPU:
a single-precision evaluation of the same sums stays inside them, and one
wrong output value does not."""
import numpy as np
import pytest

import oracle
import siggen
from gpu_util import check_ddc_elements, check_pfb_elements, f32


def _pfb_fp32(h, N, M, iq):
    """FP32 fold (M-term sums of FP32 products) and a single-precision FFT."""
    x = np.asarray(iq, np.float32).reshape(-1, 2)
    xc = (x[:, 0] + 1j * x[:, 1]).astype(np.complex64)
    h32 = np.asarray(h, np.float32)
    F = oracle.pfb_nframes(xc.size, N, M)
    v = np.zeros((F, N), np.complex64)
    for m in range(M):
        blk = np.stack([xc[(p + m) * N:(p + m + 1) * N] for p in range(F)])
        v = (v + blk * h32[m * N:(m + 1) * N]).astype(np.complex64)
    return np.fft.fft(v, axis=1).astype(np.complex64)


@pytest.mark.parametrize("N,M", [(64, 4), (256, 8)])
def test_pfb_bound_holds_and_catches_one_bin(N, M):
    h = siggen.pfb_prototype(N, M, "kaiser", 9.0)
    spec = siggen.StreamSpec(11, siggen.pfb_small().stream.tones, 700.0)
    n = N * M + 40 * N
    iq = spec.iq(0, n)
    ref = oracle.pfb(f32(h), N, M, iq=iq)
    y = _pfb_fp32(h, N, M, iq)
    assert check_pfb_elements(y, ref, h, N, M, iq) < 0.5
    bad = y.copy()
    f, k = 17, N // 3
    bad[f, k] += np.float32(np.abs(ref[f]).mean())      # one bin off by a typical bin's size
    with pytest.raises(AssertionError):
        check_pfb_elements(bad, ref, h, N, M, iq)


def test_ddc_bound_holds_and_catches_one_output():
    rng = np.random.default_rng(4)
    T, D, n, nt = 256, 100, 6000, 5
    words = siggen.random_words(rng, nt)
    phi0 = siggen.random_words(rng, nt)
    h = siggen.ddc_lowpass(T, 80e3 * 4, win="blackman")
    spec = siggen.StreamSpec(31, siggen.ToneSet(words, np.full(nt, 40.0), rng.uniform(0, 6.28, nt)), 300.0)
    iq = spec.iq(0, n)
    ref = oracle.ddc(words, phi0, f32(h), D, iq=iq)
    # the same sums in FP32: FP32 products h x times the table's values rounded to FP32
    x = np.asarray(iq, np.float32).reshape(-1, 2)
    xc = (x[:, 0] + 1j * x[:, 1]).astype(np.complex64)
    tab = oracle.nco_table().astype(np.complex64)
    hr = np.asarray(h, np.float32)[::-1]
    y = np.zeros_like(ref, dtype=np.complex64)
    for t in range(nt):
        for o in range(ref.shape[1]):
            ph = np.array([oracle.nco_phase(int(phi0[t]), int(words[t]), o * D + j) for j in range(T)], np.uint64)
            c = np.conj(tab[(ph >> np.uint64(48)).astype(np.int64)])
            u = (xc[o * D:o * D + T] * hr).astype(np.complex64)
            y[t, o] = np.sum((u * c).astype(np.complex64), dtype=np.complex64)
    assert check_ddc_elements(y, ref, f32(h), D, iq) < 0.5
    bad = y.copy()
    bad[2, 7] += np.float32(np.abs(ref[2]).mean())
    with pytest.raises(AssertionError):
        check_ddc_elements(bad, ref, f32(h), D, iq)
