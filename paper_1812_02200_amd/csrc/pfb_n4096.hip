// Instantiations of the fused PFB kernel for N = 4096 (M = 1..16), all bins or
// chosen channels.
#include "pfb_kernels.hpp"

namespace rfk {

hipError_t launch_pfb_n4096(const PfbLaunch &a, hipStream_t s)
{
    if (a.sel) return launch_pfb_nv<4096, 8>(a, s);
    return launch_pfb_nv<4096, 0>(a, s);
}

hipError_t launch_pfb_group_n4096(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    return launch_pfb_group_n<4096>(M, hdr, items, grid, s);
}

const void *pfb_group_fn_n4096(int M)
{
    return pfb_group_fn<4096>(M);
}

}  // namespace rfk
