"""Pins of the FP64 oracle against facts fixed outside it (CPU only).

Each test checks the oracle against something the paper or mathematics fixes:
brute force on tiny inputs, a library routine, a closed form, an invariant, or
a special case.  They are chosen so that a dropped term, a wrong sign or index,
or a transposed operand anywhere in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
import siggen

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pins.json")))
RNG = np.random.default_rng(12345)


def crand(*shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def relerr(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def hhat(h, omega):
    """DTFT of the taps, sum_r h[r] exp(-i omega r), by direct summation."""
    r = np.arange(h.size)
    return np.sum(h * np.exp(-1j * omega * r))


# ----------------------------------------------------------- P1, P2: DFT stage

@pytest.mark.parametrize("N", [1, 2, 4, 8, 16, 64, 256])
def test_p1_fft_matches_direct_dft(N):
    x = crand(N)
    assert relerr(oracle.fft_pow2(x), oracle.dft_direct(x)) < 1e-13


@pytest.mark.parametrize("N", [3, 12, 100])
def test_p1_direct_dft_matches_brute_force_matrix(N):
    # brute force with the DFT matrix built from numpy's exp
    x = crand(N)
    n = np.arange(N)
    W = np.exp(-2j * np.pi * np.outer(n, n) / N)
    assert relerr(oracle.dft_direct(x), W @ x) < 1e-12


@pytest.mark.parametrize("N,M", [(4, 1), (8, 2), (16, 4), (64, 4)])
def test_p1_pfb_dft_stage_is_direct_dft_of_fold(N, M):
    x = crand(N * (M + 5) + 3)
    h = RNG.standard_normal(N * M)
    X = oracle.pfb(h, N, M, x=x)
    V = oracle.pfb_fold(h, N, M, x=x)
    ref = np.array([oracle.dft_direct(v) for v in V])
    assert relerr(X, ref) < 1e-12


@pytest.mark.parametrize("N,M", [(64, 4), (256, 8), (1024, 2), (60, 3), (1000, 2), (1536, 1)])
def test_p2_pfb_dft_stage_matches_numpy_fft(N, M):
    # powers of two go through the oracle's FFT, other N through its direct sum
    x = crand(N * (M + 3))
    h = RNG.standard_normal(N * M)
    X = oracle.pfb(h, N, M, x=x)
    V = oracle.pfb_fold(h, N, M, x=x)
    assert relerr(X, np.fft.fft(V, axis=1)) < (1e-13 if N & (N - 1) == 0 else 1e-12)


@pytest.mark.parametrize("N,M", [(1024, 4), (6000, 2), (100000, 1)])
def test_p2_fold_fft_matches_direct_dft_at_sampled_bins(N, M):
    # pfb_fold_fft (fold + numpy FFT, the full-spectrum reference for large N)
    # against the oracle's direct DFT sum at sampled bins, and, for a power of
    # two, against the oracle's own radix-2 path at every bin
    iq = np.clip(np.rint(RNG.normal(0, 900, 2 * N * (M + 2))), -8192, 8191).astype(np.int16)
    h = RNG.standard_normal(N * M)
    X = oracle.pfb_fold_fft(h, N, M, iq=iq)
    bins = np.unique(np.concatenate([RNG.integers(0, N, 12), [0, 1, N // 2, N - 1]]))
    assert relerr(X[:, bins], oracle.pfb_channels(h, N, M, bins, iq=iq)) < 1e-11
    if N & (N - 1) == 0:
        assert relerr(X, oracle.pfb(h, N, M, iq=iq)) < 1e-13
    # Parseval on every frame: sum_k |X_p[k]|^2 = N sum_n |v_p[n]|^2
    V = oracle.pfb_fold(h, N, M, iq=iq)
    assert np.allclose(np.sum(np.abs(X) ** 2, 1), N * np.sum(np.abs(V) ** 2, 1), rtol=1e-12)


def test_p2_fold_brute_force_tiny():
    # N=4, M=3: v_p[n] = sum_m h[mN+n] x[pN+mN+n] written out for p = 1
    N, M = 4, 3
    x = crand(N * 6)
    h = RNG.standard_normal(N * M)
    V = oracle.pfb_fold(h, N, M, x=x)
    p = 1
    want = [h[n] * x[p * N + n] + h[N + n] * x[p * N + N + n] + h[2 * N + n] * x[p * N + 2 * N + n]
            for n in range(N)]
    assert np.allclose(V[p], want, rtol=0, atol=1e-13)


# ------------------------------------------------- P3: block DFT special case

@pytest.mark.parametrize("N", [16, 64, 512])
def test_p3_single_tap_all_ones_is_block_dft(N):
    x = crand(N * 20)
    X = oracle.pfb(np.ones(N), N, 1, x=x)
    assert X.shape == (20, N)
    assert relerr(X, np.fft.fft(x.reshape(-1, N), axis=1)) < 1e-13
    # Parseval: sum |X|^2 = N sum |x|^2
    assert np.isclose(np.sum(np.abs(X) ** 2), N * np.sum(np.abs(x) ** 2), rtol=1e-12)


# ------------------------------------- P4: impulse fixes tap order and alignment

@pytest.mark.parametrize("N,M", [(8, 3), (16, 4)])
@pytest.mark.parametrize("amp", [1000, 1000j])
def test_p4_impulse_response(N, M, amp):
    S = N * (M + 6)
    h = RNG.standard_normal(N * M)
    k = np.arange(N)
    for r0 in [0, 1, N - 1, N + 3, 3 * N + 5, S - 1]:
        x = np.zeros(S, dtype=np.complex128)
        x[r0] = amp
        # int16 input carries I at even, Q at odd indices
        iq = siggen.quantize(x)
        X = oracle.pfb(h, N, M, iq=iq)
        assert X.shape[0] == (S - N * M) // N + 1
        for p in range(X.shape[0]):
            d = r0 - p * N
            if 0 <= d < N * M:
                want = amp * h[d] * np.exp(-2j * np.pi * k * d / N)
            else:
                want = np.zeros(N)
            assert np.allclose(X[p], want, rtol=0, atol=1e-9 * abs(amp)), (r0, p)


# ------------------------- P5, P6: bin-centred and half-bin tones (prototype)

def tone(N, k0, A, theta, S):
    m = np.arange(S)
    return A * np.exp(1j * (2 * np.pi * k0 * m / N + theta))


@pytest.mark.parametrize("N,M,win", [(64, 4, "hann"), (256, 8, "kaiser")])
def test_p5_bin_centred_tone_lands_in_one_channel(N, M, win):
    h = siggen.pfb_prototype(N, M, win, 9.0)
    A, theta, k0 = 1234.5, 0.7, 5
    x = tone(N, k0, A, theta, N * (M + 7))
    X = oracle.pfb(h, N, M, x=x)
    # the tone's channel carries A e^{i theta} times the DC gain (sum h = 1)
    assert np.allclose(X[:, k0], A * np.exp(1j * theta) * h.sum(), rtol=1e-12, atol=0)
    assert np.isclose(h.sum(), 1.0, rtol=1e-14)
    # every other channel equals A e^{i theta} Hhat(2 pi (k - k0) / N)
    for kk in [0, k0 - 1, k0 + 1, k0 + 2, N - 1]:
        want = A * np.exp(1j * theta) * hhat(h, 2 * np.pi * (kk - k0) / N)
        assert np.allclose(X[:, kk], want, rtol=0, atol=1e-9 * A)


@pytest.mark.parametrize("N,M,win,adj_db", [(64, 4, "hann", -44.4), (1024, 8, "kaiser", -93.6)])
def test_p5_adjacent_channel_rejection(N, M, win, adj_db):
    # adjacent-channel rejection of the two prototypes, computed in FP64 from the
    # taps' DTFT independently of the oracle; the oracle's output must show it
    h = siggen.pfb_prototype(N, M, win, 9.0)
    x = tone(N, 3, 1.0, 0.0, N * (M + 1))
    X = oracle.pfb(h, N, M, x=x)
    got = 20 * np.log10(np.abs(X[0, 4]))
    assert abs(got - adj_db) < 0.1
    assert np.isclose(np.abs(X[0, 4]), np.abs(hhat(h, 2 * np.pi / N)), rtol=1e-6)


@pytest.mark.parametrize("N,M,win,want_db", [(64, 4, "hann", -6.117), (1024, 8, "kaiser", -6.021)])
def test_p6_half_bin_tone_crosses_at_6db(N, M, win, want_db):
    pin = GOLDEN["pfb_adjacent_crosstalk_db"]
    h = siggen.pfb_prototype(N, M, win, 9.0)
    k0 = 7
    x = tone(N, k0 + 0.5, 1.0, 0.3, N * (M + 2))
    X = oracle.pfb(h, N, M, x=x)
    a, b = np.abs(X[:, k0]), np.abs(X[:, k0 + 1])
    assert np.allclose(a, b, rtol=1e-9)                 # symmetric prototype
    db = 20 * np.log10(a)
    assert np.all(np.abs(db - pin["value"]) < pin["tolerance_db"])   # paper: about 6 dB
    assert np.all(np.abs(db - want_db) < 0.01)


# ------------------------------------------------------------ P7: linearity

def test_p7_pfb_linearity():
    N, M = 32, 4
    h = RNG.standard_normal(N * M)
    x, y = crand(N * 12), crand(N * 12)
    a, b = 2.5 - 1j, -0.75 + 3j
    lhs = oracle.pfb(h, N, M, x=a * x + b * y)
    rhs = a * oracle.pfb(h, N, M, x=x) + b * oracle.pfb(h, N, M, x=y)
    assert relerr(lhs, rhs) < 1e-13


def test_p7_pfb_linearity_int16_exact_sum():
    N, M = 64, 4
    w = siggen.pfb_small(nsamples=N * 40)
    rng = np.random.default_rng(7)
    a = rng.integers(-3000, 3000, size=2 * N * 40).astype(np.int16)
    b = rng.integers(-3000, 3000, size=2 * N * 40).astype(np.int16)
    s = (a.astype(np.int32) + b).astype(np.int16)   # exact: no overflow
    lhs = oracle.pfb(w.h, N, M, iq=s)
    rhs = oracle.pfb(w.h, N, M, iq=a) + oracle.pfb(w.h, N, M, iq=b)
    assert relerr(lhs, rhs) < 1e-13


def test_p7_ddc_linearity():
    words = np.array([123456789123456789, 2**63 + 5, 17], dtype=np.uint64)
    h = siggen.ddc_lowpass(40, 3e6)
    x, y = crand(400), crand(400)
    a, b = 1.5, -2j
    lhs = oracle.ddc(words, None, h, 7, x=a * x + b * y)
    rhs = a * oracle.ddc(words, None, h, 7, x=x) + b * oracle.ddc(words, None, h, 7, x=y)
    assert relerr(lhs, rhs) < 1e-13


# ------------------------------- P8: time-shift covariance (frame/output index)

def test_p8_pfb_shift_by_whole_frames():
    N, M, q = 16, 4, 3
    h = RNG.standard_normal(N * M)
    x = crand(N * 30)
    full = oracle.pfb(h, N, M, x=x)
    part = oracle.pfb(h, N, M, x=x[q * N:])
    assert np.array_equal(part, full[q:])
    sel = oracle.pfb(h, N, M, x=x, frames=[5, 0, 26])
    assert np.array_equal(sel, full[[5, 0, 26]])
    assert np.isnan(oracle.pfb(h, N, M, x=x, frames=[27])).all()


def test_p8_ddc_shift_by_whole_outputs():
    words = np.array([987654321987654321, 3 * 2**61 + 11], dtype=np.uint64)
    phi0 = np.array([5, 2**64 - 3], dtype=np.uint64)
    h = siggen.ddc_lowpass(30, 5e6)
    D, q = 9, 4
    x = crand(500)
    full = oracle.ddc(words, phi0, h, D, x=x)
    # start q*D samples later: the NCO must start at phi0 + q*D*inc
    phi_q = np.array([oracle.nco_phase(int(p), int(w), q * D) for p, w in zip(phi0, words)],
                     dtype=np.uint64)
    part = oracle.ddc(words, phi_q, h, D, x=x[q * D:])
    assert np.allclose(part, full[:, q:], rtol=0, atol=1e-12)
    pts = oracle.ddc_points(words, phi0, h, D, [1, 0, 1], [0, 3, full.shape[1] - 1], x=x)
    assert np.allclose(pts, [full[1, 0], full[0, 3], full[1, -1]], rtol=0, atol=1e-12)


# ------------------------------------------ P9: the paper's moving average

def test_p9_boxcar_is_conjugate_phase_times_mean():
    D = 500   # paper Sec. III.B: decimation 500 with a moving average
    ntones = 5
    rng = np.random.default_rng(9)
    iq = rng.integers(-8192, 8192, size=2 * (D * 6 + 123)).astype(np.int16)
    phi0 = rng.integers(0, 2**64, size=ntones, dtype=np.uint64)
    words = np.zeros(ntones, dtype=np.uint64)
    y = oracle.ddc(words, phi0, siggen.boxcar(D), D, iq=iq)
    assert y.shape == (ntones, 6)
    tab = np.exp(2j * np.pi * np.arange(65536) / 65536)
    I = iq[0::2].astype(np.int64)
    Q = iq[1::2].astype(np.int64)
    for n in range(6):
        mean = (I[n * D:(n + 1) * D].sum() + 1j * Q[n * D:(n + 1) * D].sum()) / D  # exact sums
        for t in range(ntones):
            want = np.conj(tab[int(phi0[t]) >> 48]) * mean
            assert abs(y[t, n] - want) < 1e-9


# ------------------------------------- P10: exact-frequency tone gives DC

def test_p10_on_grid_tone_is_constant_dc():
    T, D = 64, 16
    h = siggen.ddc_lowpass(T, 2e6)
    A, theta = 777.0, -1.1
    for kidx in [0, 1, 12345, 65535]:
        w = np.uint64(kidx) << np.uint64(48)
        m = np.arange(T * 8)
        x = A * np.exp(1j * (2 * np.pi * kidx * m / 65536.0 + theta))
        y = oracle.ddc(np.array([w]), None, h, D, x=x)
        assert np.allclose(y, A * np.exp(1j * theta) * h.sum(), rtol=1e-12, atol=0)


def test_p10_off_grid_tone_within_truncation_bound():
    T, D = 128, 32
    h = siggen.ddc_lowpass(T, 1e6)
    A, theta = 1000.0, 0.25
    words = siggen.random_words(np.random.default_rng(10), 6)
    for w in words:
        m = np.arange(T * 6, dtype=np.uint64)
        ang = (m * w).astype(np.float64) * (2 * np.pi / 2.0**64)
        x = A * np.exp(1j * (ang + theta))
        y = oracle.ddc(np.array([w]), None, h, D, x=x)
        # truncating the phase to 16 bits errs by < 2 pi / 2^16 rad per sample
        assert np.all(np.abs(y - A * np.exp(1j * theta)) <= A * 2 * np.pi / 65536)
        ye = oracle.ddc(np.array([w]), None, h, D, x=x, exact_nco=True)
        assert np.allclose(ye, A * np.exp(1j * theta), rtol=0, atol=1e-9 * A)


# ------------------------------------- P15-P17: chirped NCO (Sec. III.C, Eq. 1)

def _eq1_cycles_exact(f0, k, fs, m):
    """Eq. 1's phase in cycles, f0 t + k t^2 at t = m/fs, as an exact rational."""
    from fractions import Fraction
    t = Fraction(m) / Fraction(fs)
    return Fraction(f0) * t + Fraction(k) * t * t


def test_p15_chirp_phase_is_eq1_exactly_for_dyadic_parameters():
    # f0/fs and k/fs^2 dyadic: the words are exact and the integer phase must
    # equal 2^64 (f0 t + k t^2) mod 2^64 at every sample, however large m is.
    # A ramp read as k (not 2k) or an m^2 term in place of m(m-1)/2 fails.
    fs = 2.0**28
    for f0, k in [(3 * 2.0**20, 5 * 2.0**30), (-(2.0**25), 2.0**33), (0.0, -(7 * 2.0**29))]:
        inc, K = siggen.chirp_words(f0, k, fs)
        for m in [0, 1, 2, 3, 1000, 123457, 2**33 + 5, 2**40 + 17]:
            want = _eq1_cycles_exact(f0, k, fs, m) * 2**64
            assert want.denominator == 1
            assert oracle.chirp_phase(0, inc, K, m) == int(want) % 2**64


def test_p15_chirp_phase_rounding_bound_for_arbitrary_parameters():
    # Rounded words: |phase - 2^64 Eq.1| <= m/2 + m(m-1)/4 + 1 (the two word
    # roundings, each at most 1/2, times m and m(m-1)/2).
    rng = np.random.default_rng(15)
    for _ in range(20):
        f0 = float(rng.uniform(-90e6, 90e6))
        k = float(rng.uniform(-5e12, 5e12))
        inc, K = siggen.chirp_words(f0, k)
        for m in [1, 17, 4096, 10**6, 3 * 10**7]:
            want = _eq1_cycles_exact(f0, k, siggen.FS, m) * 2**64
            d = (oracle.chirp_phase(0, inc, K, m) - round(want)) % 2**64
            d = d - 2**64 if d >= 2**63 else d
            assert abs(d) <= m / 2 + m * (m - 1) / 4 + 1


def test_p16_chirp_closed_form_equals_second_order_accumulator():
    rng = np.random.default_rng(16)
    for _ in range(5):
        p0, inc, K = (int(v) for v in rng.integers(0, 2**64, size=3, dtype=np.uint64))
        phi, rate = p0, inc
        for m in range(3000):
            assert oracle.chirp_phase(p0, inc, K, m) == phi
            phi = (phi + rate) % 2**64
            rate = (rate + K) % 2**64
        assert oracle.chirp_phase(p0, inc, 0, 987654321) == oracle.nco_phase(p0, inc, 987654321)


def test_p17_ddc_of_matching_chirp_is_constant_dc():
    # Input: an unquantised chirp A exp(i (2 pi phi[m]/2^64 + theta)); the DDC
    # tone follows the same chirp, so every output is A exp(i theta) sum(h),
    # exactly with the untruncated NCO and within the 16-bit phase truncation
    # bound with the table.
    T, D = 96, 40
    h = siggen.ddc_lowpass(T, 1e6)
    A, theta = 900.0, 0.7
    for f0, k in [(12.5e6, 3e12), (-40e6, -8e12), (77e6, 2.5e13)]:
        inc, K = siggen.chirp_words(f0, k)
        m0 = 5_000_000                       # start late in the chirp: large quadratic term
        S = T + 7 * D
        ph = np.array([oracle.chirp_phase(0, inc, K, m0 + m) for m in range(S)], dtype=np.uint64)
        x = A * np.exp(1j * (ph.astype(np.float64) * (2 * np.pi / 2.0**64) + theta))
        # the stream starts at m0: the tone's phase at local sample 0 is phi(m0)
        # and its rate is inc + K m0
        p0 = np.array([oracle.chirp_phase(0, inc, K, m0)], dtype=np.uint64)
        inc0 = np.array([(inc + K * m0) % 2**64], dtype=np.uint64)
        y = oracle.ddc(inc0, p0, h, D, x=x, chirp=np.array([K], dtype=np.uint64))
        assert y.shape == (1, 8)
        assert np.all(np.abs(y - A * np.exp(1j * theta) * h.sum()) <= A * np.abs(h).sum() * 2 * np.pi / 65536)
        ye = oracle.ddc(inc0, p0, h, D, x=x, chirp=np.array([K], dtype=np.uint64), exact_nco=True)
        assert np.allclose(ye, A * np.exp(1j * theta) * h.sum(), rtol=0, atol=1e-9 * A)
        # with the linear NCO (K dropped) the chirp walks out of the passband
        yl = oracle.ddc(inc0, p0, h, D, x=x)
        assert np.abs(yl).min() < 0.1 * A


def test_p17_zero_chirp_is_the_linear_nco():
    rng = np.random.default_rng(17)
    w = siggen.random_words(rng, 5)
    p0 = siggen.random_words(rng, 5)
    h = siggen.ddc_lowpass(64, 2e6)
    iq = siggen.quantize(rng.normal(0, 900, size=3000) + 1j * rng.normal(0, 900, size=3000))
    a = oracle.ddc(w, p0, h, 25, iq=iq)
    b = oracle.ddc(w, p0, h, 25, iq=iq, chirp=np.zeros(5, dtype=np.uint64))
    assert np.array_equal(a, b)


# ----------------------------------------------- P11, P12: NCO phase and table

def test_p11_nco_phase_closed_form_bit_exact():
    rng = np.random.default_rng(11)
    for _ in range(200):
        p0 = int(rng.integers(0, 2**64, dtype=np.uint64))
        inc = int(rng.integers(0, 2**64, dtype=np.uint64))
        m = int(rng.integers(0, 2**40))
        assert oracle.nco_phase(p0, inc, m) == (p0 + m * inc) % 2**64   # Python big integers
    words = rng.integers(0, 2**64, size=50, dtype=np.uint64)
    p0s = rng.integers(0, 2**64, size=50, dtype=np.uint64)
    S = 134217728
    got = oracle.nco_phases(words, p0s, S)
    want = [(int(a) + S * int(b)) % 2**64 for a, b in zip(p0s, words)]
    assert [int(g) for g in got] == want


def test_p12_nco_table():
    tab = oracle.nco_table()
    assert tab[0] == 1 + 0j
    assert abs(tab[16384] - 1j) < 1e-15 and abs(tab[32768] + 1) < 1e-15
    i = np.arange(65536)
    assert np.allclose(tab, np.cos(2 * np.pi * i / 65536) + 1j * np.sin(2 * np.pi * i / 65536),
                       rtol=0, atol=2e-16)
    # quarter-wave symmetry: Tab[i + 2^14] = i * Tab[i]
    assert np.allclose(tab[16384:], 1j * tab[:-16384], rtol=0, atol=1e-15)


# --------------------------------------------------- P13: DDC == PFB bin

@pytest.mark.parametrize("N,M", [(16, 4), (64, 4)])
def test_p13_ddc_equals_pfb_channel(N, M):
    w = siggen.pfb_small(nsamples=N * 50)
    h = siggen.pfb_prototype(N, M, "hann")
    iq = siggen.StreamSpec(5, w.stream.tones, 800.0).iq(0, N * 50)
    X = oracle.pfb(h, N, M, iq=iq)
    words = np.array([k * (2**64 // N) for k in range(N)], dtype=np.uint64)
    Y = oracle.ddc(words, None, h[::-1].copy(), N, iq=iq)
    assert Y.shape == (N, X.shape[0])
    assert relerr(Y.T, X) < 1e-12


# ------------------------------------------------ counts fixed by the workloads

def test_output_counts():
    for key in ("pfb_small_frames", "pfb_production_frames"):
        g = GOLDEN[key]
        assert oracle.pfb_nframes(g["nsamples"], g["N"], g["M"]) == g["value"]
    g = GOLDEN["ddc_bank_outputs"]
    assert oracle.ddc_noutputs(g["nsamples"], g["T"], g["D"]) == g["value"]
    assert oracle.pfb_nframes(255, 64, 4) == 0 and oracle.pfb_nframes(256, 64, 4) == 1
    assert oracle.ddc_noutputs(1023, 1024, 1000) == 0 and oracle.ddc_noutputs(1024, 1024, 1000) == 1


def test_pfb_small_workload_end_to_end_properties():
    # the parity workload's 8 bin-centred tones dominate their channels
    w = siggen.pfb_small()
    iq = w.stream.iq(0, w.nsamples)
    X = oracle.pfb(w.h, w.N, w.M, iq=iq, frames=np.arange(0, 16381, 97))
    bins = sorted(int(round(int(t) * w.N / 2.0**64)) % w.N for t in w.stream.tones.words)
    p = np.mean(np.abs(X) ** 2, axis=0)
    top = sorted(np.argsort(p)[-8:])
    assert top == bins


# ------------------------------------------- P18-P22: Tx synthesis (DAC buffers)

def test_p18_tab32_is_the_fp32_table_with_exact_symmetry():
    t = oracle.tab32().astype(np.float64)
    i = np.arange(65536)
    a = 2 * np.pi * i / 65536.0
    # each entry is the FP32 rounding of the true value (within half an FP32 ulp)
    assert np.abs(t[:, 0] - np.cos(a)).max() <= 2.0**-25 * 1.0001
    assert np.abs(t[:, 1] - np.sin(a)).max() <= 2.0**-25 * 1.0001
    # quarter-turn and half-turn symmetry, exactly
    assert np.array_equal(t[(i + 16384) % 65536, 0], -t[i, 1])
    assert np.array_equal(t[(i + 16384) % 65536, 1], t[i, 0])
    assert np.array_equal(t[(i + 32768) % 65536], -t[i])
    # the same values as the DDC oracle's FP64 table rounded to FP32, but for rare ties
    ref = oracle.nco_table()
    ref32 = np.stack([ref.real, ref.imag], axis=1).astype(np.float32).astype(np.float64)
    assert np.mean(t == ref32) > 0.999


def _tx_numpy(phase, rate, chirp, amp, n):
    """Independent reference: numpy FP32 scalars, tones in ascending order."""
    tab = oracle.tab32()
    out = np.empty(2 * n, dtype=np.int16)
    for j in range(n):
        vr = np.float32(0.0)
        vi = np.float32(0.0)
        for t in range(len(phase)):
            tri = j * (j - 1) // 2
            ph = (int(phase[t]) + j * int(rate[t]) + int(chirp[t]) * tri) % 2**64
            c = tab[ph >> 48]
            vr = np.float32(vr + np.float32(np.float32(amp[t]) * c[0]))
            vi = np.float32(vi + np.float32(np.float32(amp[t]) * c[1]))
        for k, v in enumerate((vr, vi)):
            r = np.rint(v)
            out[2 * j + k] = int(min(max(r, -32768.0), 32767.0))
    return out


def test_p19_tx_matches_independent_fp32_reference():
    rng = np.random.default_rng(19)
    nt, n = 6, 400
    phase = siggen.random_words(rng, nt)
    rate = siggen.random_words(rng, nt)
    chirp = siggen.random_words(rng, nt)
    chirp[:3] = 0
    amp = rng.uniform(-9000, 9000, nt).astype(np.float32)
    amp[0] = 30000.0                          # drives some samples into saturation
    got = oracle.tx(phase, rate, amp, n, chirp=chirp)
    assert np.array_equal(got, _tx_numpy(phase, rate, chirp, amp, n))
    assert got.max() == 32767 or got.min() == -32768


def test_p20_tx_then_ddc_recovers_the_amplitude():
    # A tone generated at amplitude A and demodulated with the same oscillator
    # gives A sum(h) |Tab|^2 plus the DAC rounding error (<= 0.5 LSB per
    # component): |y - A sum h| <= A 2^-23 sum|h| + sqrt(2)/2 sum|h|.
    rng = np.random.default_rng(20)
    T = D = 1024
    h = siggen.boxcar(D)
    for A in [100.0, 2345.5, 31000.0]:
        w = int(siggen.random_words(rng, 1)[0])
        p0 = int(siggen.random_words(rng, 1)[0])
        iq = oracle.tx([p0], [w], [A], 8 * D)
        y = oracle.ddc([w], [p0], h, D, iq=iq)[0]
        assert y.size == 8
        assert np.all(np.abs(y - A) <= A * 2.0**-23 + np.sqrt(2) / 2)


def test_p21_tx_bin_centred_tones_in_the_spectrum():
    N = 1024
    bins = np.array([3, 100, 257, 511, 700, 1000])
    amps = np.array([4000.0, 100.0, 2500.0, 800.0, 3333.0, 50.0], dtype=np.float32)
    words = (bins.astype(np.uint64) << np.uint64(54))   # bin k of N = 2^10: k * 2^64 / 2^10
    iq = oracle.tx(np.zeros(6, np.uint64), words, amps, N)
    x = iq[0::2].astype(np.float64) + 1j * iq[1::2]
    X = np.fft.fft(x)
    # each tone's bin carries N*A (the DAC rounding adds at most N * 0.71 LSB)
    assert np.all(np.abs(np.abs(X[bins]) - N * amps) <= N * 0.71)
    rest = np.delete(np.abs(X), bins)
    assert rest.max() <= N * 0.71


def test_p22_tx_buffers_continue_the_waveform():
    rng = np.random.default_rng(22)
    nt = 9
    phase = siggen.random_words(rng, nt)
    rate = siggen.random_words(rng, nt)
    chirp = siggen.random_words(rng, nt)
    amp = rng.uniform(-3000, 3000, nt).astype(np.float32)
    whole = oracle.tx(phase, rate, amp, 5000, chirp=chirp)
    parts, ph, rt = [], phase, rate
    for n in [1, 0, 777, 2, 2220]:
        parts.append(oracle.tx(ph, rt, amp, n, chirp=chirp))
        ph, rt = oracle.tx_advance(ph, rt, n, chirp=chirp)
    parts.append(oracle.tx(ph, rt, amp, 5000 - 3000, chirp=chirp))
    assert np.array_equal(np.concatenate(parts), whole)
    # the advanced state is the closed form at sample n
    ph2, rt2 = oracle.tx_advance(phase, rate, 12345, chirp=chirp)
    for t in range(nt):
        assert int(ph2[t]) == oracle.chirp_phase(int(phase[t]), int(rate[t]), int(chirp[t]), 12345)
        assert int(rt2[t]) == (int(rate[t]) + 12345 * int(chirp[t])) % 2**64


def test_p22_tx_chirp_is_demodulated_by_the_chirped_ddc():
    # Eq. 1 chirp generated as a DAC buffer, demodulated with the same words.
    inc, K = siggen.chirp_words(-30e6, 9e12)
    A = 5000.0
    T, D = 256, 200
    h = siggen.ddc_lowpass(T, 1e6)
    iq = oracle.tx([0], [inc], [A], T + 20 * D, chirp=[K])
    y = oracle.ddc([inc], None, h, D, iq=iq, chirp=[K])[0]
    assert np.all(np.abs(y - A * h.sum()) <= A * 2.0**-23 * np.abs(h).sum() + np.sqrt(2) / 2 * np.abs(h).sum())


# ----------------------------------------------- P23: selected channels (Sec. III.A)

@pytest.mark.parametrize("N,M", [(16, 4), (64, 8), (256, 2)])
def test_p23_selected_channels_equal_the_full_spectrum_columns(N, M):
    # the direct evaluation at chosen bins agrees with the FFT path's columns
    rng = np.random.default_rng(N + M)
    h = siggen.pfb_prototype(N, M, "kaiser", 9.0)
    iq = siggen.quantize(rng.normal(0, 2000, 40 * N) + 1j * rng.normal(0, 2000, 40 * N))
    chans = rng.choice(N, size=min(N, 11), replace=False)
    chans = np.concatenate([chans, [0, N - 1, N // 2]])
    chans = np.unique(chans)[rng.permutation(np.unique(chans).size)]
    full = oracle.pfb(h, N, M, iq=iq)
    sub = oracle.pfb_channels(h, N, M, chans, iq=iq)
    assert sub.shape == (full.shape[0], chans.size)
    assert np.allclose(sub, full[:, chans], rtol=0, atol=1e-9 * np.abs(full).max())
