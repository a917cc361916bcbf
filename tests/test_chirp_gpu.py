"""GPU parity of chirped DDC banks (ddc_create_chirp; paper Sec. III.C, Eq. 1)
against the FP64 oracle.

Same bar as the ordinary DDC: FP32 outputs within RMS 1e-5 of a full-scale
tone's output, the 64-bit phase bit-exact after every call (closed form
phi0 + S inc + K S(S-1)/2 mod 2^64), results independent of how the stream is
cut into buffers (bit for bit), and a zero chirp reproducing the ordinary bank
bit for bit.
"""
import numpy as np
import pytest

import oracle
import siggen
from gpu_util import check_ddc_elements, err_fs, err_rel, f32, log, need_gpu, run_ddc, to_dev

pytestmark = pytest.mark.gpu

TOL_FS = 1e-5
TOL_REL = 1e-6


def tol_rel(T):
    return TOL_REL * np.sqrt(max(T, 1024) / 1024.0)


def _rf():
    need_gpu()
    import paper_1812_02200_amd as rf
    return rf


def chirp_bank(rng, ntones):
    """Eq. 1 chirps (f0 within +-90 MHz, k within +-2e13 Hz/s) and, for every
    fifth tone, arbitrary 64-bit words."""
    inc = np.empty(ntones, dtype=np.uint64)
    K = np.empty(ntones, dtype=np.uint64)
    for t in range(ntones):
        if t % 5 == 4:
            inc[t], K[t] = (int(v) for v in rng.integers(0, 2**64, size=2, dtype=np.uint64))
        else:
            inc[t], K[t] = siggen.chirp_words(float(rng.uniform(-90e6, 90e6)), float(rng.uniform(-2e13, 2e13)))
    return inc, K


def phases_after(inc, phi0, K, S):
    p0 = np.zeros_like(inc) if phi0 is None else phi0
    return np.array([oracle.chirp_phase(int(a), int(b), int(c), S) for a, b, c in zip(p0, inc, K)],
                    dtype=np.uint64)


CASES = [
    # ntones, T, D, nsamples
    (1, 1, 1, 300),
    (9, 5, 3, 1000),
    (64, 64, 16, 5000),
    (300, 1024, 1000, 50000),
    (1100, 256, 200, 20000),      # more tones than one work-group
    (20, 1500, 700, 12000),       # filter longer than one LDS chunk
    (12, 10, 37, 3000),           # decimation larger than the filter
]


@pytest.mark.parametrize("ntones,T,D,n", CASES)
def test_chirp_parity(ntones, T, D, n):
    rf = _rf()
    import torch
    rng = np.random.default_rng(ntones * 11 + T)
    inc, K = chirp_bank(rng, ntones)
    phi0 = siggen.random_words(rng, ntones)
    h = siggen.ddc_lowpass(T, 80e3 * 1024 / max(T, 1), win="blackman") if T > 1 else np.ones(1)
    iq = siggen.StreamSpec(53, siggen.ToneSet(siggen.random_words(rng, 20), np.full(20, 60.0),
                                              rng.uniform(0, 6.28, 20)), 300.0).iq(0, n)
    log("chirp parity tones=%d T=%d D=%d n=%d" % (ntones, T, D, n))
    dd = rf.Ddc(inc, h, D, phi0, max_samples_per_call=n, chirp=K)
    y = run_ddc(dd, to_dev(iq), [n], torch)
    ref = oracle.ddc(inc, phi0, f32(h), D, iq=iq, chirp=K)
    assert y.shape == ref.shape
    e, r = err_fs(y, ref, h.sum()), err_rel(y, ref)
    log("  err_fs=%.3g err_rel=%.3g" % (e, r))
    assert e <= TOL_FS and r <= tol_rel(T)
    check_ddc_elements(y, ref, f32(h), D, iq)
    assert np.array_equal(dd.phase(), phases_after(inc, phi0, K, n))


@pytest.mark.parametrize("ntones,T,D", [(100, 1024, 1000), (7, 10, 37), (64, 100, 1)])
def test_chirp_split_invariance_and_phase(ntones, T, D):
    rf = _rf()
    import torch
    rng = np.random.default_rng(3 * T + D)
    inc, K = chirp_bank(rng, ntones)
    h = siggen.ddc_lowpass(T, 1e6)
    n = 40000
    iq = siggen.StreamSpec(59, siggen.ToneSet(inc[:8], np.full(min(8, ntones), 100.0),
                                              np.zeros(min(8, ntones))), 200.0).iq(0, n)
    d = to_dev(iq)
    whole = run_ddc(rf.Ddc(inc, h, D, max_samples_per_call=n, chirp=K), d, [n], torch)
    dd = rf.Ddc(inc, h, D, max_samples_per_call=n, chirp=K)
    sizes, pos = [], 0
    for c in [0, 1, 2, T - 1, D + 1, 0, 3 * D + 7] + list(rng.integers(1, 3 * max(T, D), 200)):
        c = int(min(c, n - pos))
        sizes.append(c)
        pos += c
        if pos == n:
            break
    if pos < n:
        sizes.append(n - pos)
    outs, pos = [], 0
    for s in sizes:
        no = dd.outputs_for(s)
        out = torch.empty((ntones, max(no, 1)), dtype=torch.complex64, device="cuda")
        outs.append(dd.process(d[2 * pos: 2 * (pos + s)], out=out))
        pos += s
        if s:
            assert np.array_equal(dd.phase(), phases_after(inc, None, K, pos))
    got = torch.cat(outs, 1).cpu().numpy()
    assert got.shape == whole.shape
    assert np.array_equal(got.view(np.uint64), whole.view(np.uint64))


def test_zero_chirp_is_the_ordinary_bank_bit_exact():
    rf = _rf()
    import torch
    rng = np.random.default_rng(61)
    words = siggen.random_words(rng, 257)
    phi0 = siggen.random_words(rng, 257)
    h = siggen.ddc_lowpass(300, 2e6)
    n = 25000
    d = to_dev(siggen.StreamSpec(61, siggen.ToneSet(words[:9], np.full(9, 80.0), np.zeros(9)), 250.0).iq(0, n))
    a = run_ddc(rf.Ddc(words, h, 120, phi0, max_samples_per_call=n), d, [n], torch)
    z = rf.Ddc(words, h, 120, phi0, max_samples_per_call=n, chirp=np.zeros(257, dtype=np.uint64))
    b = run_ddc(z, d, [n], torch)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert np.array_equal(z.phase(), oracle.nco_phases(words, phi0, n))


def test_chirp_state_resume_and_fingerprint():
    rf = _rf()
    import torch
    rng = np.random.default_rng(67)
    inc, K = chirp_bank(rng, 150)
    phi0 = siggen.random_words(rng, 150)
    h = siggen.ddc_lowpass(200, 2e6)
    D, n, cut = 150, 30011, 12345
    d = to_dev(siggen.StreamSpec(67, siggen.ToneSet(inc[:10], np.full(10, 50.0), np.zeros(10)), 250.0).iq(0, n))
    whole = run_ddc(rf.Ddc(inc, h, D, phi0, max_samples_per_call=n, chirp=K), d, [n], torch)
    b = rf.Ddc(inc, h, D, phi0, max_samples_per_call=n, chirp=K)
    first = run_ddc(b, d[: 2 * cut], [cut], torch)
    blob = b.get_state()
    c = rf.Ddc(inc, h, D, phi0, max_samples_per_call=n, chirp=K)
    c.set_state(blob)
    assert np.array_equal(c.phase(), phases_after(inc, phi0, K, cut))
    second = run_ddc(c, d[2 * cut:], [n - cut], torch)
    got = np.concatenate([first, second], axis=1)
    assert np.array_equal(got.view(np.uint64), whole.view(np.uint64))
    # a bank with other chirp words (or none) refuses the blob
    K2 = K.copy()
    K2[3] ^= np.uint64(1)
    for other in (rf.Ddc(inc, h, D, phi0, max_samples_per_call=n, chirp=K2),
                  rf.Ddc(inc, h, D, phi0, max_samples_per_call=n)):
        with pytest.raises(rf.RfError):
            other.set_state(blob)


def test_matched_chirp_demodulates_to_constant_dc():
    """A quantised Eq. 1 chirp (amplitude 3000 LSB) demodulated by a tone with
    the same words: every output equals 3000 exp(i theta) sum(h) up to the
    16-bit phase truncation and the input quantisation (<= 0.5 LSB per
    component), on the GPU as in the oracle."""
    rf = _rf()
    import torch
    T, D, n = 512, 400, 60000
    A, theta = 3000.0, 0.3
    h = siggen.ddc_lowpass(T, 1e6)
    for f0, k in [(15e6, 4e12), (-60e6, 1.5e13)]:
        inc, K = siggen.chirp_words(f0, k)
        ph = np.array([oracle.chirp_phase(0, inc, K, m) for m in range(n)], dtype=np.uint64)
        x = A * np.exp(1j * (ph.astype(np.float64) * (2 * np.pi / 2.0**64) + theta))
        iq = siggen.quantize(x)
        dd = rf.Ddc([inc], h, D, max_samples_per_call=n, chirp=[K])
        y = run_ddc(dd, to_dev(iq), [n], torch)[0]
        want = A * np.exp(1j * theta) * h.sum()
        bound = A * np.abs(h).sum() * 2 * np.pi / 65536 + np.sqrt(2) * 0.5 * np.abs(h).sum()
        assert np.all(np.abs(y - want) <= bound)
        ref = oracle.ddc([inc], None, f32(h), D, iq=iq, chirp=[K])[0]
        assert err_fs(y, ref, h.sum()) <= TOL_FS


@pytest.mark.slow
def test_chirp_bank_full_size_sampled():
    """1000 chirped tones, T=1024 Blackman, D=1000, 2^27 samples in 2^23 buffers:
    phases bit-exact, sampled outputs (buffer edges included) against the oracle."""
    rf = _rf()
    import torch
    w = siggen.ddc_bank()
    rng = np.random.default_rng(71)
    inc, K = chirp_bank(rng, 1000)
    d = siggen.iq_torch(w.stream, 0, w.nsamples)
    torch.cuda.synchronize()
    dd = rf.Ddc(inc, w.h, w.D, w.phase0, max_samples_per_call=w.buffer, chirp=K)
    total = 134217
    out = torch.empty((1000, total), dtype=torch.complex64, device="cuda")
    pos, o, bounds = 0, 0, []
    sh = torch.cuda.current_stream().cuda_stream
    while pos < w.nsamples:
        got = dd.process_ptr(d.data_ptr() + 4 * pos, w.buffer, out.data_ptr() + 8 * o, total, sh)
        bounds.append(o)
        o += got
        pos += w.buffer
    torch.cuda.synchronize()
    assert o == total
    assert np.array_equal(dd.phase(), phases_after(inc, w.phase0, K, w.nsamples))
    outs = sorted(set([0, total - 1] + bounds + [b - 1 for b in bounds if b > 0]))
    ti = np.concatenate([rng.integers(0, 1000, len(outs)), rng.integers(0, 1000, 150)])
    oi = np.concatenate([outs, rng.integers(0, total, 150)])
    y = out.cpu().numpy()[ti, oi]
    iq = d.cpu().numpy()
    ref = oracle.ddc_points(inc, w.phase0, f32(w.h), w.D, ti, oi, iq=iq, chirp=K)
    e, r = err_fs(y, ref, w.h.sum()), err_rel(y, ref)
    log("  err_fs=%.3g err_rel=%.3g" % (e, r))
    assert e <= TOL_FS and r <= tol_rel(1024)
    check_ddc_elements(y, ref, f32(w.h), w.D, iq, tones=ti, outs=oi)
