// Instantiations of the fused PFB kernel for N = 32 (M = 1..16), all bins or
// chosen channels.
#include "pfb_kernels.hpp"

namespace rfk {

hipError_t launch_pfb_n32(const PfbLaunch &a, hipStream_t s)
{
    if (a.sel) return launch_pfb_nv<32, 8>(a, s);
    return launch_pfb_nv<32, 0>(a, s);
}

hipError_t launch_pfb_group_n32(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    return launch_pfb_group_n<32>(M, hdr, items, grid, s);
}

const void *pfb_group_fn_n32(int M)
{
    return pfb_group_fn<32>(M);
}

}  // namespace rfk
