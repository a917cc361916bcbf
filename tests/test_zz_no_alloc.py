"""pfb_process_static (the process call that allocates nothing) against
pfb_process: the same stream fed to two handles, one through each call, on
two calls in a row (the second smaller), must give bit-identical spectra; a
call whose scratch would exceed the static array is refused and leaves the
handle unchanged.
"""
import numpy as np
import pytest

import oracle
import siggen
from gpu_util import err_rel, f32, log, need_gpu

pytestmark = pytest.mark.gpu

STATIC_BYTES = 64 << 20


def _rf():
    need_gpu()
    import paper_1812_02200_amd as rf
    return rf


def _stream(n, seed, N):
    rng = np.random.default_rng(seed)
    words = np.array([siggen.bin_word(k + 0.25 * (k % 4), N) for k in rng.integers(0, N, 8)], dtype=np.uint64)
    tones = siggen.ToneSet(words, np.full(8, 500.0), rng.uniform(0, 6.28, 8))
    return siggen.StreamSpec(seed, tones, 600.0).iq(0, n)


def _feed(p, d, sizes, static, torch):
    """Feed d in calls of the given sizes through pfb_process or
    pfb_process_static; returns the frames of each call (numpy)."""
    s = torch.cuda.current_stream().cuda_stream
    outs, pos = [], 0
    for n in sizes:
        F = p.frames_for(n)
        out = torch.empty((max(F, 1), p.N), dtype=torch.complex64, device="cuda")
        call = p.process_static_ptr if static else p.process_ptr
        got = call(d.data_ptr() + 4 * pos, n, out.data_ptr(), max(F, 1), s)
        assert got == F
        outs.append(out[:F])
        pos += n
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in outs]


@pytest.mark.parametrize("N,M,first,second", [
    (100000, 4, 100000 * 4 + 30 * 100000 + 17, 5 * 100000 + 3),   # two-step plan, 200 x 500
    (3000, 3, 3000 * 3 + 600 * 3000 + 11, 40 * 3000 + 7),          # one-step plan
    (1024, 8, 1024 * 8 + 900 * 1024 + 5, 77 * 1024 + 1),           # fused kernel, no scratch
])
def test_static_scratch_matches_process(N, M, first, second):
    rf = _rf()
    import torch
    h = siggen.pfb_prototype(N, M, "kaiser", 9.0)
    n = first + second
    iq = _stream(n, N + M, N)
    d = torch.from_numpy(iq).cuda()
    a = rf.Pfb(N, M, h, max_samples_per_call=first)
    b = rf.Pfb(N, M, h, max_samples_per_call=first)
    log("no-alloc N=%d M=%d calls of %d then %d samples" % (N, M, first, second))
    ya = _feed(a, d, [first, second], False, torch)
    yb = _feed(b, d, [first, second], True, torch)
    for k in range(2):
        assert ya[k].shape == yb[k].shape
        assert np.array_equal(ya[k].view(np.uint64), yb[k].view(np.uint64)), k
    assert a.counters() == b.counters()
    got = np.concatenate(yb)
    ref = oracle.pfb_fold_fft(f32(h), N, M, iq=iq)
    assert got.shape == ref.shape
    r = err_rel(got, ref)
    log("  bit-identical to pfb_process; err_rel vs oracle %.3g" % r)
    assert r <= 1e-6


def test_static_scratch_refuses_oversized_calls():
    rf = _rf()
    import torch
    N, M = 100000, 2
    h = siggen.pfb_prototype(N, M, "kaiser", 9.0)
    big = N * M + 60 * N             # 61 frames: 2 x 61 x 10^5 x 8 B > 64 MiB
    small = N * M + 10 * N + 99
    n = big + small
    iq = _stream(n, 5, N)
    d = torch.from_numpy(iq).cuda()
    p = rf.Pfb(N, M, h, max_samples_per_call=big)
    assert 2 * p.frames_for(big) * N * 8 > STATIC_BYTES
    out = torch.empty((p.frames_for(big), N), dtype=torch.complex64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    with pytest.raises(rf.RfError) as ei:
        p.process_static_ptr(d.data_ptr(), big, out.data_ptr(), out.shape[0], s)
    assert ei.value.status == rf.RF_EINVAL
    assert p.counters() == (0, 0, 0)
    # the handle is unchanged: a fitting call still matches pfb_process
    q = rf.Pfb(N, M, h, max_samples_per_call=big)
    yq = _feed(q, d, [small], False, torch)
    yp = _feed(p, d, [small], True, torch)
    assert np.array_equal(yq[0].view(np.uint64), yp[0].view(np.uint64))
