"""Chosen PFB channels (pfb_set_channels; paper Sec. III.A, full spectrum or
specific user-defined channels) on the GPU.

The transform is the same as for the full spectrum, so the chosen channels
must equal the corresponding bins of the full output bit for bit; against
the oracle (a direct DFT at the chosen bins) the FP32 bar of the PFB applies.
"""
import numpy as np
import pytest

import oracle
import siggen
from gpu_util import check_pfb_elements, err_fs, f32, log, need_gpu, run_pfb, to_dev

pytestmark = pytest.mark.gpu


def _rf():
    need_gpu()
    import paper_1812_02200_amd as rf
    return rf


def stream(N, M, n, seed):
    rng = np.random.default_rng(seed)
    tones = siggen.ToneSet(siggen.random_words(rng, 16), np.full(16, 400.0), rng.uniform(0, 6.28, 16))
    return siggen.StreamSpec(seed, tones, 900.0).iq(0, n)


@pytest.mark.parametrize("N,M", [(16, 1), (64, 4), (256, 8), (1024, 8), (4096, 4)])
def test_chosen_channels_are_the_full_spectrum_columns(N, M):
    rf = _rf()
    import torch
    rng = np.random.default_rng(N * 3 + M)
    h = siggen.pfb_prototype(N, M, "kaiser", 9.0)
    n = N * M + 37 * N + 7
    iq = stream(N, M, n, N + M)
    d = to_dev(iq)
    full = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), d, [n], torch)
    for chans in (rng.permutation(N)[: max(1, N // 7)], np.array([N - 1]), np.arange(N)[::-1].copy(),
                  np.array([0, N // 2, 1, N - 1])):
        log("channels N=%d M=%d nsel=%d" % (N, M, chans.size))
        p = rf.Pfb(N, M, h, max_samples_per_call=n)
        p.set_channels(chans)
        got = run_pfb(p, d, [n], torch)
        assert got.shape == (full.shape[0], chans.size)
        assert np.array_equal(got.view(np.uint64), full[:, chans].view(np.uint64))
    ch = rng.permutation(N)[: min(N, 9)]
    ref = oracle.pfb_channels(f32(h), N, M, ch, iq=iq)
    p = rf.Pfb(N, M, h, max_samples_per_call=n)
    p.set_channels(ch)
    got = run_pfb(p, d, [n], torch)
    assert err_fs(got, ref, h.sum()) <= 1e-5
    check_pfb_elements(got, ref, h, N, M, iq)


def test_chosen_channels_across_buffers_and_switches():
    rf = _rf()
    import torch
    N, M = 1024, 8
    h = siggen.pfb_prototype(N, M, "kaiser", 9.0)
    n = 200 * N + 333
    iq = stream(N, M, n, 5)
    d = to_dev(iq)
    full = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), d, [n], torch)
    rng = np.random.default_rng(5)
    ch = rng.permutation(N)[:16]
    p = rf.Pfb(N, M, h, max_samples_per_call=n)
    p.set_channels(ch)
    sizes = [N * M - 1, 1, 5 * N + 3, 0, 77 * N, n]
    outs, pos, fr = [], 0, 0
    for i, s in enumerate(sizes):
        s = min(s, n - pos)
        if i == 3:
            p.set_channels(None)             # full spectrum for a while
        if i == 4:
            p.set_channels(ch)
        y = run_pfb(p, d[2 * pos: 2 * (pos + s)], [s], torch)
        want = full[fr: fr + y.shape[0]]
        want = want if p.width == N else want[:, ch]
        assert np.array_equal(y.view(np.uint64), want.view(np.uint64))
        pos += s
        fr += y.shape[0]
    assert fr == full.shape[0]


def test_channel_choice_is_validated():
    rf = _rf()
    h = siggen.pfb_prototype(64, 4)
    p = rf.Pfb(64, 4, h)
    for bad in ([64], [-1], [3, 5, 3]):
        with pytest.raises(rf.RfError):
            p.set_channels(bad)
    assert p.width == 64
    m = rf.Pfb(256, 4, siggen.pfb_prototype(256, 4), dft_mode=rf.RF_DFT_MFMA_F16X2)
    with pytest.raises(rf.RfError) as ei:
        m.set_channels([1, 2])
    assert ei.value.status == rf.RF_EUNSUPPORTED
