// Instantiations of the MFMA DFT PFB kernel for N = 256 (M = 1..16, FP16 and BF16).
#include "pfb_mfma.hpp"

namespace rfk {

hipError_t launch_pfb_mfma_n256(const PfbLaunch &a, int prec, hipStream_t s) { return launch_mfma_n<256>(a, prec, s); }

}  // namespace rfk
