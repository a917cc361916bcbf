"""CPU-side checks of the C-ABI library: it loads, exports every declared call,
and rejects invalid arguments before touching the device.  No compute call is
made here (there is no GPU on this tier)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1812_02200_amd as rf
from paper_1812_02200_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rfchan.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_documented_calls():
    names = declared_functions()
    for must in ["pfb_create", "pfb_process", "ddc_create", "ddc_process", "rf_strerror",
                 "pfb_frames_for", "ddc_outputs_for", "ddc_get_phase", "ddc_create_chirp",
                 "tx_create", "tx_synthesize", "tx_set_tones", "tx_get_state"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = rf.lib()
    names = declared_functions()
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", rf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if l.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # the binding declares exactly the header's calls
    assert sorted(_lib.SIGNATURES) == names


def test_status_strings():
    lib = rf.lib()
    for code in range(7):
        assert lib.rf_strerror(code)
    assert lib.rf_strerror(0) == b"ok"
    assert rf.version() >= 100


def _pfb_create(N, M, proto, mode=0, maxs=1024):
    h = ctypes.c_void_p()
    arr = None if proto is None else np.ascontiguousarray(proto, dtype=np.float32)
    st = rf.lib().pfb_create(ctypes.byref(h), N, M, None if arr is None else arr.ctypes.data, mode, maxs)
    return st, h


# 1001 = 7 * 11 * 13 and 4097 = 17 * 241 have other prime factors; 2^25 is too
# large; 3^15 has no split into two factors <= 4096.
@pytest.mark.parametrize("N,M", [(1001, 4), (8, 4), (4097, 1), (1 << 25, 1), (3 ** 15, 1),
                                 (64, 0), (64, 17), (0, 1)])
def test_pfb_create_rejects_bad_shapes(N, M):
    st, h = _pfb_create(N, M, np.zeros(max(min(N * M, 1 << 20), 1)))
    assert st == rf.RF_EINVAL and not h.value
    assert rf.lib().rf_last_error()


def test_large_n_split_rules():
    # products of 2, 3 and 5 up to 2^24 that split into two factors <= 4096
    # are accepted by the validation (creation then needs a device)
    for N in (100, 1000, 6000, 100000, 10**6, 10**7, 8192, 1 << 24):
        st, h = _pfb_create(N, 2, np.zeros(2 * N))
        assert st != rf.RF_EINVAL, N
    for N, mode in ((1000, rf.RF_DFT_MFMA_F16X2), (100000, rf.RF_DFT_MFMA_BF16X2)):
        st, h = _pfb_create(N, 2, np.zeros(1), mode=mode)
        assert st == rf.RF_EUNSUPPORTED


def test_pfb_create_rejects_bad_arguments():
    assert _pfb_create(64, 4, None)[0] == rf.RF_EINVAL
    assert _pfb_create(64, 4, np.zeros(256), maxs=0)[0] == rf.RF_EINVAL
    assert _pfb_create(64, 4, np.zeros(256), mode=9)[0] == rf.RF_EINVAL
    bad = np.zeros(256)
    bad[3] = np.nan
    assert _pfb_create(64, 4, bad)[0] == rf.RF_EINVAL
    assert rf.lib().pfb_create(None, 64, 4, None, 0, 1) == rf.RF_EINVAL


def test_ddc_create_rejects_bad_arguments():
    lib = rf.lib()
    inc = np.arange(4, dtype=np.uint64)
    taps = np.ones(8, np.float32)
    h = ctypes.c_void_p()
    assert lib.ddc_create(ctypes.byref(h), 0, inc.ctypes.data, None, 8, taps.ctypes.data, 2, 10) == rf.RF_EINVAL
    assert lib.ddc_create(ctypes.byref(h), 4, None, None, 8, taps.ctypes.data, 2, 10) == rf.RF_EINVAL
    assert lib.ddc_create(ctypes.byref(h), 4, inc.ctypes.data, None, 0, taps.ctypes.data, 2, 10) == rf.RF_EINVAL
    assert lib.ddc_create(ctypes.byref(h), 4, inc.ctypes.data, None, 5000, taps.ctypes.data, 2, 10) == rf.RF_EINVAL
    assert lib.ddc_create(ctypes.byref(h), 4, inc.ctypes.data, None, 8, taps.ctypes.data, 0, 10) == rf.RF_EINVAL
    assert lib.ddc_create(ctypes.byref(h), 4, inc.ctypes.data, None, 8, None, 2, 10) == rf.RF_EINVAL
    assert not h.value


def test_ddc_create_chirp_and_tx_create_reject_bad_arguments():
    lib = rf.lib()
    inc = np.arange(4, dtype=np.uint64)
    K = np.arange(4, dtype=np.uint64)
    taps = np.ones(8, np.float32)
    amp = np.ones(4, np.float32)
    h = ctypes.c_void_p()
    assert lib.ddc_create_chirp(ctypes.byref(h), 0, inc.ctypes.data, None, K.ctypes.data, 8,
                                taps.ctypes.data, 2, 10) == rf.RF_EINVAL
    assert lib.ddc_create_chirp(ctypes.byref(h), 4, None, None, K.ctypes.data, 8,
                                taps.ctypes.data, 2, 10) == rf.RF_EINVAL
    assert lib.tx_create(ctypes.byref(h), 0, inc.ctypes.data, None, None, amp.ctypes.data, 10) == rf.RF_EINVAL
    assert lib.tx_create(ctypes.byref(h), 4, None, None, None, amp.ctypes.data, 10) == rf.RF_EINVAL
    assert lib.tx_create(ctypes.byref(h), 4, inc.ctypes.data, None, None, None, 10) == rf.RF_EINVAL
    assert lib.tx_create(ctypes.byref(h), 4, inc.ctypes.data, None, None, amp.ctypes.data, 0) == rf.RF_EINVAL
    bad = amp.copy()
    bad[2] = np.inf
    assert lib.tx_create(ctypes.byref(h), 4, inc.ctypes.data, None, None, bad.ctypes.data, 10) == rf.RF_EINVAL
    assert not h.value


def test_null_handles_are_rejected():
    lib = rf.lib()
    assert lib.pfb_frames_for(None, 100) == 0
    assert lib.ddc_outputs_for(None, 100) == 0
    assert lib.pfb_process(None, None, 0, None, 0, None, None) == rf.RF_EINVAL
    assert lib.ddc_process(None, None, 0, None, 0, None, None) == rf.RF_EINVAL
    assert lib.pfb_destroy(None) == rf.RF_OK and lib.ddc_destroy(None) == rf.RF_OK
    assert lib.pfb_reset(None) == rf.RF_EINVAL and lib.ddc_reset(None) == rf.RF_EINVAL
    assert lib.tx_synthesize(None, None, 0, None) == rf.RF_EINVAL
    assert lib.tx_set_tones(None, None, None, None) == rf.RF_EINVAL
    assert lib.tx_get_state(None, None, None, None) == rf.RF_EINVAL
    assert lib.tx_reset(None) == rf.RF_EINVAL and lib.tx_destroy(None) == rf.RF_OK


def test_python_binding_raises_instead_of_falling_back():
    with pytest.raises(rf.RfError):
        rf.Pfb(100, 4, np.zeros(400))
    with pytest.raises(ValueError):
        rf.Pfb(64, 4, np.zeros(10))


def test_stream_footprint_counts_staging_slots_and_eight_column_taps():
    """Admission arithmetic (host only): pinned-host staging slots add
    host_slots x max_buffer x 4 bytes; the N = 4096 eight-column kernel's
    per-thread tap copy doubles the taps; output slots scale the output part."""
    h = np.zeros(1024 * 8, np.float32)
    d0, _ = rf.Server.make_desc(pfb=(1024, 8, h), max_buffer=1 << 20, out_slots=2)
    d3, _ = rf.Server.make_desc(pfb=(1024, 8, h), max_buffer=1 << 20, out_slots=2, host_slots=3)
    assert rf.Server.footprint(d3) - rf.Server.footprint(d0) == 3 * (1 << 20) * 4
    d1, _ = rf.Server.make_desc(pfb=(1024, 8, h), max_buffer=1 << 20, out_slots=1)
    frames = ((1024 * 8 + (1 << 20)) // 1024 + 1)
    assert rf.Server.footprint(d0) - rf.Server.footprint(d1) == frames * 1024 * 8
    h4 = np.zeros(4096 * 8, np.float32)
    h2 = np.zeros(2048 * 8, np.float32)
    f4, _ = rf.Server.make_desc(pfb=(4096, 8, h4), max_buffer=1 << 20, out_slots=1)
    f2, _ = rf.Server.make_desc(pfb=(2048, 8, h2), max_buffer=1 << 20, out_slots=1)
    # state beyond the output slot: taps (x2 at N = 4096), twiddles, two histories
    s4 = rf.Server.footprint(f4) - ((4096 * 8 + (1 << 20)) // 4096 + 1) * 4096 * 8
    s2 = rf.Server.footprint(f2) - ((2048 * 8 + (1 << 20)) // 2048 + 1) * 2048 * 8
    assert s4 - 4 * 4096 * 8 * 4 > 0 and s2 - 3 * 2048 * 8 * 4 > 0
    assert s4 >= 4 * 4096 * 8 * 4 and s2 < 4 * 2048 * 8 * 4
