"""GPU parity of the DDC bank (ddc_* C ABI) against the FP64 oracle.

Bar: FP32 outputs within RMS 1e-5 of a full-scale tone's output (8192 * sum h),
the 64-bit NCO phase bit-exact after every call, and as a regression guard
||e||/||y_ref|| <= 1e-6 * sqrt(max(T, 1024) / 1024): each output is an FP32 sum of
T products whose rounding error grows like sqrt(T), while noise-dominated
outputs are much smaller than the sum of the magnitudes of their terms.
"""
import numpy as np
import pytest

import oracle
import siggen
from gpu_util import check_ddc_elements, err_fs, err_rel, f32, log, need_gpu, run_ddc, run_pfb, to_dev

pytestmark = pytest.mark.gpu

TOL_FS = 1e-5
TOL_REL = 1e-6


def tol_rel(T):
    return TOL_REL * np.sqrt(max(T, 1024) / 1024.0)


def _rf():
    need_gpu()
    import paper_1812_02200_amd as rf
    return rf


CASES = [
    # ntones, T, D, nsamples
    (1, 1, 1, 300),
    (7, 3, 2, 1000),
    (64, 64, 16, 5000),
    (100, 256, 200, 1 << 15),
    (1000, 1024, 1000, 50000),
    (1500, 512, 300, 20000),      # more tones than one work-group
    (33, 4096, 1024, 20000),      # longest filter
    (10, 10, 37, 3000),           # decimation larger than the filter: samples are skipped
]


@pytest.mark.parametrize("ntones,T,D,n", CASES)
def test_ddc_parity(ntones, T, D, n):
    rf = _rf()
    import torch
    rng = np.random.default_rng(ntones * 7 + T)
    words = siggen.random_words(rng, ntones)
    phi0 = siggen.random_words(rng, ntones)
    h = siggen.ddc_lowpass(T, 80e3 * 1024 / max(T, 1), win="blackman") if T > 1 else np.ones(1)
    spec = siggen.StreamSpec(31, siggen.ToneSet(words[:50], np.full(min(ntones, 50), 40.0),
                                                rng.uniform(0, 6.28, min(ntones, 50))), 300.0)
    iq = spec.iq(0, n)
    log("ddc parity tones=%d T=%d D=%d n=%d" % (ntones, T, D, n))
    dd = rf.Ddc(words, h, D, phi0, max_samples_per_call=n)
    y = run_ddc(dd, to_dev(iq), [n], torch)
    ref = oracle.ddc(words, phi0, f32(h), D, iq=iq)
    assert y.shape == ref.shape
    e, r = err_fs(y, ref, h.sum()), err_rel(y, ref)
    log("  err_fs=%.3g err_rel=%.3g" % (e, r))
    assert e <= TOL_FS and r <= tol_rel(T)
    check_ddc_elements(y, ref, f32(h), D, iq)
    assert np.array_equal(dd.phase(), oracle.nco_phases(words, phi0, n))


@pytest.mark.parametrize("ntones,T,D", [(100, 1024, 1000), (5, 10, 37), (64, 100, 1)])
def test_ddc_split_invariance_and_phase(ntones, T, D):
    rf = _rf()
    import torch
    rng = np.random.default_rng(T + D)
    words = siggen.random_words(rng, ntones)
    h = siggen.ddc_lowpass(T, 1e6)
    n = 40000
    iq = siggen.StreamSpec(37, siggen.ToneSet(words[:8], np.full(min(8, ntones), 100.0),
                                              np.zeros(min(8, ntones))), 200.0).iq(0, n)
    d = to_dev(iq)
    whole = run_ddc(rf.Ddc(words, h, D, max_samples_per_call=n), d, [n], torch)
    dd = rf.Ddc(words, h, D, max_samples_per_call=n)
    sizes, pos = [], 0
    cuts = [0, 1, 2, T - 1, D + 1, 0, 3 * D + 7]
    for c in cuts + list(rng.integers(1, 3 * max(T, D), 200)):
        c = int(min(c, n - pos))
        sizes.append(c)
        pos += c
        if pos == n:
            break
    if pos < n:
        sizes.append(n - pos)
    outs = []
    pos = 0
    for s in sizes:
        no = dd.outputs_for(s)
        out = torch.empty((ntones, max(no, 1)), dtype=torch.complex64, device="cuda")
        y = dd.process(d[2 * pos: 2 * (pos + s)], out=out)
        pos += s
        outs.append(y)
        if s:
            assert np.array_equal(dd.phase(), oracle.nco_phases(words, None, pos))
    got = torch.cat(outs, 1).cpu().numpy()
    assert got.shape == whole.shape
    assert np.array_equal(got.view(np.uint64), whole.view(np.uint64))


def test_ddc_state_resume_and_reset():
    rf = _rf()
    import torch
    rng = np.random.default_rng(41)
    words = siggen.random_words(rng, 300)
    phi0 = siggen.random_words(rng, 300)
    h = siggen.ddc_lowpass(200, 2e6)
    D = 150
    n = 30011
    iq = siggen.StreamSpec(41, siggen.ToneSet(words[:20], np.full(20, 50.0), np.zeros(20)), 250.0).iq(0, n)
    d = to_dev(iq)
    a = rf.Ddc(words, h, D, phi0, max_samples_per_call=n)
    whole = run_ddc(a, d, [n], torch)
    cut = 12345
    b = rf.Ddc(words, h, D, phi0, max_samples_per_call=n)
    first = run_ddc(b, d[: 2 * cut], [cut], torch)
    blob = b.get_state()
    c = rf.Ddc(words, h, D, phi0, max_samples_per_call=n)
    c.set_state(blob)
    assert np.array_equal(c.phase(), b.phase())
    second = run_ddc(c, d[2 * cut:], [n - cut], torch)
    got = np.concatenate([first, second], axis=1)
    assert np.array_equal(got.view(np.uint64), whole.view(np.uint64))
    a.reset()
    assert np.array_equal(a.phase(), phi0)
    again = run_ddc(a, d, [n], torch)
    assert np.array_equal(again.view(np.uint64), whole.view(np.uint64))
    other = rf.Ddc(words[::-1].copy(), h, D, phi0, max_samples_per_call=n)
    with pytest.raises(rf.RfError):
        other.set_state(blob)


def test_ddc_paper_moving_average_workload():
    """Paper Sec. III.B: ~200 tones, moving-average filter, decimation 500, at 100 Msps."""
    rf = _rf()
    import torch
    rng = np.random.default_rng(43)
    fs = 100e6
    freqs = rng.uniform(-45e6, 45e6, 200)
    words = np.array([siggen.tuning_word(f, fs) for f in freqs], dtype=np.uint64)
    h = siggen.boxcar(500)
    n = 500 * 40 + 321
    spec = siggen.StreamSpec(43, siggen.ToneSet(words, np.full(200, 30.0), rng.uniform(0, 6.28, 200)), 100.0)
    iq = spec.iq(0, n)
    dd = rf.Ddc(words, h, 500, max_samples_per_call=n)
    y = run_ddc(dd, to_dev(iq), [n], torch)
    ref = oracle.ddc(words, None, f32(h), 500, iq=iq)
    assert y.shape == (200, 40)
    assert err_fs(y, ref, h.sum()) <= TOL_FS and err_rel(y, ref) <= TOL_REL


def test_ddc_matches_pfb_channels_on_gpu():
    """A bin-centred DDC with D = N, T = N*M and the reversed prototype is the PFB."""
    rf = _rf()
    import torch
    N, M = 256, 8
    h = siggen.pfb_prototype(N, M, "kaiser")
    n = N * 80 + 17
    iq = siggen.StreamSpec(47, siggen.pfb_small().stream.tones, 600.0).iq(0, n)
    d = to_dev(iq)
    X = run_pfb(rf.Pfb(N, M, h, max_samples_per_call=n), d, [n], torch)
    words = np.array([k * (2**64 // N) for k in range(N)], dtype=np.uint64)
    Y = run_ddc(rf.Ddc(words, h[::-1].copy(), N, max_samples_per_call=n), d, [n], torch)
    assert Y.shape == (N, X.shape[0])
    assert err_fs(Y.T, X, h.sum()) <= TOL_FS
    assert err_rel(Y.T, X) <= 2 * TOL_REL


def test_ddc_on_grid_tone_is_dc():
    rf = _rf()
    import torch
    T, D = 512, 100
    h = siggen.ddc_lowpass(T, 1e6)
    kidx = 12345
    words = np.array([np.uint64(kidx) << np.uint64(48)], dtype=np.uint64)
    tones = siggen.ToneSet(words, np.array([4000.0]), np.array([0.9]))
    n = 20000
    iq = siggen.StreamSpec(53, tones, 0.0).iq(0, n)
    y = run_ddc(rf.Ddc(words, h, D, max_samples_per_call=n), to_dev(iq), [n], torch)
    want = 4000.0 * np.exp(0.9j) * f32(h).sum()
    # int16 quantisation noise only: well below 1 LSB
    assert np.max(np.abs(y - want)) < 1.0


def test_ddc_tune_keeps_results_bit_exact(tmp_path, monkeypatch):
    monkeypatch.setenv("RFCHAN_TUNE_CACHE", str(tmp_path / "tune.txt"))
    rf = _rf()
    import torch
    rng = np.random.default_rng(59)
    words = siggen.random_words(rng, 700)
    h = siggen.ddc_lowpass(512, 1e6)
    n = 60000
    iq = siggen.StreamSpec(59, siggen.ToneSet(words[:10], np.full(10, 40.0), np.zeros(10)), 300.0).iq(0, n)
    d = to_dev(iq)
    base = run_ddc(rf.Ddc(words, h, 400, max_samples_per_call=n), d, [n], torch)
    dd = rf.Ddc(words, h, 400, max_samples_per_call=n)
    us, grid = dd.tune(n)
    assert us > 0 and grid >= 1
    got = run_ddc(dd, d, [n], torch)
    assert np.array_equal(got.view(np.uint64), base.view(np.uint64))
    assert rf.Ddc(words, h, 400, max_samples_per_call=n).apply_tuned(n)


@pytest.mark.slow
def test_ddc_bank_full_size_sampled():
    """1000 tones, T=1024 Blackman, D=1000, 2^27 samples in 2^23 buffers -> 1000 x 134217.

    All phases bit-exact; sampled outputs (buffer edges included) against the oracle.
    """
    rf = _rf()
    import torch
    w = siggen.ddc_bank()
    log("ddc bank: generating 2^27 samples on the device")
    d = siggen.iq_torch(w.stream, 0, w.nsamples)
    torch.cuda.synchronize()
    dd = rf.Ddc(w.words, w.h, w.D, w.phase0, max_samples_per_call=w.buffer)
    total = 134217
    out = torch.empty((1000, total), dtype=torch.complex64, device="cuda")
    pos, o = 0, 0
    bounds = []
    sh = torch.cuda.current_stream().cuda_stream
    while pos < w.nsamples:
        got = dd.process_ptr(d.data_ptr() + 4 * pos, w.buffer, out.data_ptr() + 8 * o, total, sh)
        bounds.append(o)
        o += got
        pos += w.buffer
    torch.cuda.synchronize()
    assert o == total
    assert np.array_equal(dd.phase(), oracle.nco_phases(w.words, w.phase0, w.nsamples))
    rng = np.random.default_rng(3)
    outs = sorted(set([0, total - 1] + bounds + [b - 1 for b in bounds if b > 0]))
    ti = np.concatenate([rng.integers(0, 1000, len(outs)), rng.integers(0, 1000, 150)])
    oi = np.concatenate([outs, rng.integers(0, total, 150)])
    y = out.cpu().numpy()[ti, oi]
    iq = d.cpu().numpy()
    ref = oracle.ddc_points(w.words, w.phase0, f32(w.h), w.D, ti, oi, iq=iq)
    e, r = err_fs(y, ref, w.h.sum()), err_rel(y, ref)
    log("ddc bank sampled points=%d err_fs=%.3g err_rel=%.3g" % (len(ti), e, r))
    assert e <= TOL_FS and r <= TOL_REL
    check_ddc_elements(y, ref, f32(w.h), w.D, iq, tones=ti, outs=oi)
