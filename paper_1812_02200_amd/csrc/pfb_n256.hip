// Instantiations of the fused PFB kernel for N = 256 (M = 1..16), all bins or
// chosen channels, plus alternate run directions (variant 16) at M = 4 and 8.
#include "pfb_kernels.hpp"

namespace rfk {

hipError_t launch_pfb_n256(const PfbLaunch &a, hipStream_t s)
{
    if (a.sel) return launch_pfb_nv<256, 8>(a, s);
    if (a.variant == 16 && a.M == 4) return launch_pfb_nmv<256, 4, 16>(a, s);
    if (a.variant == 16 && a.M == 8) return launch_pfb_nmv<256, 8, 16>(a, s);
    return launch_pfb_nv<256, 0>(a, s);
}

hipError_t launch_pfb_group_n256(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    return launch_pfb_group_n<256>(M, hdr, items, grid, s);
}

const void *pfb_group_fn_n256(int M)
{
    return pfb_group_fn<256>(M);
}

}  // namespace rfk
