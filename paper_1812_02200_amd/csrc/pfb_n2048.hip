// Instantiations of the fused PFB kernel for N = 2048 (M = 1..16), all bins or
// chosen channels, plus alternate run directions (variant 16) at M = 4 and 8.
#include "pfb_kernels.hpp"

namespace rfk {

hipError_t launch_pfb_n2048(const PfbLaunch &a, hipStream_t s)
{
    if (a.sel) return launch_pfb_nv<2048, 8>(a, s);
    if (a.variant == 16 && a.M == 4) return launch_pfb_nmv<2048, 4, 16>(a, s);
    if (a.variant == 16 && a.M == 8) return launch_pfb_nmv<2048, 8, 16>(a, s);
    return launch_pfb_nv<2048, 0>(a, s);
}

hipError_t launch_pfb_group_n2048(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    return launch_pfb_group_n<2048>(M, hdr, items, grid, s);
}

const void *pfb_group_fn_n2048(int M)
{
    return pfb_group_fn<2048>(M);
}

}  // namespace rfk
