// Instantiations of the fused PFB kernel for N = 1024 (M = 1..16), all bins or
// chosen channels, plus the tunable variants of the M = 8 kernel
// (double-buffered LDS, store type, alternate run directions) and alternate
// run directions at M = 4.
#include "pfb_kernels.hpp"

namespace rfk {

hipError_t launch_pfb_n1024(const PfbLaunch &a, hipStream_t s)
{
    if (a.sel) {
        if (a.M == 8 && (a.variant & 16)) return launch_pfb_nmv<1024, 8, 24>(a, s);
        return launch_pfb_nv<1024, 8>(a, s);
    }
    if (a.M == 8) {
        switch (a.variant) {
        case 1: return launch_pfb_nmv<1024, 8, 1>(a, s);
        case 2: return launch_pfb_nmv<1024, 8, 2>(a, s);
        case 3: return launch_pfb_nmv<1024, 8, 3>(a, s);
        case 16: return launch_pfb_nmv<1024, 8, 16>(a, s);
        case 17: return launch_pfb_nmv<1024, 8, 17>(a, s);
        default: break;
        }
    }
    if (a.M == 4 && a.variant == 16) return launch_pfb_nmv<1024, 4, 16>(a, s);
    return launch_pfb_nv<1024, 0>(a, s);
}

hipError_t launch_pfb_group_n1024(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    return launch_pfb_group_n<1024>(M, hdr, items, grid, s);
}

const void *pfb_group_fn_n1024(int M)
{
    return pfb_group_fn<1024>(M);
}

}  // namespace rfk
