"""Large and non-power-of-two channel counts (paper Sec. III.A, Fig. 3:
N = 10^5) on the GPU: fold pass + four-step FFT, against the FP64 oracle.

Full comparisons where the oracle is fast (its FFT for powers of two, its
direct DFT for N <= a few thousand); otherwise sampled bins of every frame by
the oracle's direct DFT at those bins.  Bar: RMS error <= 1e-5 of a full-scale
tone's output; buffer splits bit-identical.
"""
import numpy as np
import pytest

import oracle
import siggen
from gpu_util import err_fs, f32, log, need_gpu, run_pfb, to_dev

pytestmark = pytest.mark.gpu


def _rf():
    need_gpu()
    import paper_1812_02200_amd as rf
    return rf


def proto(N, M):
    return siggen.pfb_prototype(N, M, "kaiser", 9.0)


def stream(n, seed, N):
    rng = np.random.default_rng(seed)
    words = np.array([siggen.bin_word(k + 0.25 * (k % 4), N) for k in rng.integers(0, N, 12)], dtype=np.uint64)
    tones = siggen.ToneSet(words, np.full(12, 600.0), rng.uniform(0, 6.28, 12))
    return siggen.StreamSpec(seed, tones, 700.0).iq(0, n)


@pytest.mark.parametrize("N,M", [(60, 4), (100, 1), (1000, 8), (1536, 2), (3000, 3)])
def test_one_step_non_power_of_two_full(N, M):
    rf = _rf()
    import torch
    h = proto(N, M)
    n = N * M + 9 * N + 5
    iq = stream(n, N + M, N)
    log("large one-step N=%d M=%d" % (N, M))
    y = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), to_dev(iq), [n], torch)
    ref = oracle.pfb(f32(h), N, M, iq=iq)
    assert y.shape == ref.shape
    assert err_fs(y, ref, h.sum()) <= 1e-5


@pytest.mark.parametrize("N,M,full", [(8192, 4, True), (6000, 2, False), (100000, 8, False),
                                      (65536, 2, True), (1 << 20, 1, True)])
def test_four_step(N, M, full):
    rf = _rf()
    import torch
    h = proto(N, M)
    n = N * M + 3 * N + 11
    iq = stream(n, N % 1000 + M, N)
    log("large four-step N=%d M=%d" % (N, M))
    y = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), to_dev(iq), [n], torch)
    assert y.shape[0] == oracle.pfb_nframes(n, N, M)
    if full:
        ref = oracle.pfb(f32(h), N, M, iq=iq)
        assert err_fs(y, ref, h.sum()) <= 1e-5
    else:
        rng = np.random.default_rng(N)
        bins = np.unique(np.concatenate([rng.integers(0, N, 60), [0, 1, N - 1, N // 2]]))
        ref = oracle.pfb_channels(f32(h), N, M, bins, iq=iq)
        assert err_fs(y[:, bins], ref, h.sum()) <= 1e-5


def test_large_splits_bit_identical():
    rf = _rf()
    import torch
    N, M = 100000, 4
    h = proto(N, M)
    n = N * M + 7 * N + 123
    d = to_dev(stream(n, 7, N))
    whole = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), d, [n], torch)
    sizes = [N * M - 1, 1, 0, 2 * N + 17, N - 5, n]
    pos, tot = 0, []
    for s in sizes:
        s = min(s, n - pos)
        tot.append(s)
        pos += s
    got = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), d, tot, torch)
    assert np.array_equal(got.view(np.uint64), whole.view(np.uint64))


@pytest.mark.slow
def test_ten_million_channels_sampled():
    rf = _rf()
    import torch
    N, M = 10 ** 7, 2
    h = proto(N, M)
    n = N * M + N + 7
    iq = stream(n, 77, N)
    y = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), to_dev(iq), [n], torch)
    assert y.shape == (2, N)
    bins = np.unique(np.random.default_rng(1).integers(0, N, 24))
    ref = oracle.pfb_channels(f32(h), N, M, bins, iq=iq)
    assert err_fs(y[:, bins], ref, h.sum()) <= 1e-5


def test_fig3_shape_production_stream_sampled():
    """N = 10^5, M = 8 on the production stream in 2^24-sample buffers (the
    shape the benchmark times: hundreds of frames per call, the persistent
    step grid walking many tiles): sampled bins of every frame of the first
    2^25 samples against the oracle's direct DFT at those bins."""
    rf = _rf()
    import torch
    N, M = 100000, 8
    buf = 1 << 24
    h = proto(N, M)
    w = siggen.pfb_production()
    d = siggen.iq_torch(w.stream, 0, 2 * buf)
    p = rf.Pfb(N, M, h, max_samples_per_call=buf)
    y = run_pfb(p, d, [buf, buf], torch)
    iq = d.cpu().numpy()
    assert y.shape[0] == oracle.pfb_nframes(2 * buf, N, M)
    bins = np.unique(np.concatenate([np.random.default_rng(5).integers(0, N, 12), [0, 1, N // 2, N - 1]]))
    log("fig3 shape: %d frames, %d bins" % (y.shape[0], bins.size))
    ref = oracle.pfb_channels(f32(h), N, M, bins, iq=iq)
    assert err_fs(y[:, bins], ref, h.sum()) <= 1e-5


def test_small_non_power_of_two_with_many_frames():
    """N = 18: a buffer of 2^26 samples holds ~3.7M frames, more 32-frame
    chunks than one grid dimension covers (the fold strides over the rest);
    sampled frames, the last ones included, against the oracle at all bins."""
    rf = _rf()
    import torch
    N, M = 18, 3
    h = proto(N, M)
    n = 1 << 26
    w = siggen.pfb_small()
    d = siggen.iq_torch(w.stream, 0, n)
    y = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), d, [n], torch)
    iq = d.cpu().numpy()
    F = oracle.pfb_nframes(n, N, M)
    assert y.shape == (F, N)
    frames = np.concatenate([np.arange(64), np.arange(F - 64, F), np.random.default_rng(3).integers(0, F, 128)])
    ref = oracle.pfb(f32(h), N, M, iq=iq, frames=frames)
    assert err_fs(y[frames], ref, h.sum()) <= 1e-5
