"""MI355X-native readout channelizer and demodulator (arXiv:1812.02200 hot path).

The computation lives in librfchan.so (hand-written HIP kernels for gfx950 behind
the C ABI of include/rfchan.h); this package is its thin Python binding.
"""
from ._lib import (  # noqa: F401
    RF_DFT_FFT_F32, RF_DFT_MFMA_BF16X2, RF_DFT_MFMA_F16X2, RF_EAGAIN, RF_ECAPACITY, RF_EDEVICE,
    RF_EINVAL, RF_ENOMEM, RF_EUNSUPPORTED, RF_OK, LIB_PATH, RFS_DDC, RFS_MODE_BATCHED,
    RFS_MODE_GRAPH, RFS_MODE_SEQUENTIAL, RFS_PFB, Ddc, Pfb, RfError, Server, Tx, lib, version,
)
