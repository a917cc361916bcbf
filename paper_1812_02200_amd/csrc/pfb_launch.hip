// pfb_launch.hip -- host side of the PFB kernels: twiddle tables, default run
// length and dispatch over N.
#include <math.h>

#include "pfb_kernels.hpp"

namespace rfk {

int pfb_twiddle_count(int N)
{
    int n = 0;
    for (int ns = 4; ns < N;) {
        int R = pass_radix(N, ns);
        n += ns * R;
        ns *= R;
    }
    return n > 0 ? n : 1;
}

// Table of the pass with stride ns and radix R, at offset tw_offset(N, ns):
// entry [r][k] = exp(-2 pi i k r / (ns R)), computed in FP64, rounded to FP32.
void pfb_twiddle_fill(int N, float *tw)
{
    const double two_pi = 6.283185307179586476925286766559;
    int off = 0;
    tw[0] = 1.f;
    tw[1] = 0.f;
    for (int ns = 4; ns < N;) {
        int R = pass_radix(N, ns);
        for (int k = 0; k < ns; ++k)
            for (int r = 0; r < R; ++r) {
                long e = ((long)k * r) % ((long)ns * R);
                double ang = -two_pi * (double)e / (double)(ns * R);
                tw[2 * (off + r * ns + k)] = (float)cos(ang);
                tw[2 * (off + r * ns + k) + 1] = (float)sin(ang);
            }
        off += ns * R;
        ns *= R;
    }
}

int pfb_default_run_len(int N, int M, int64_t F)
{
    (void)N;
    (void)M;
    // Aim for about 1024 lane-group runs, between 8 and 64 frames each.
    const int64_t target = 1024;
    int64_t rl = (F + target - 1) / target;
    if (rl < 8) rl = 8;
    if (rl > 64) rl = 64;
    rl = (rl + 3) & ~3LL;
    return (int)rl;
}

hipError_t launch_pfb(const PfbLaunch &a, hipStream_t s)
{
    if (a.run_len <= 0 || (a.run_len & 3)) return hipErrorInvalidValue;
    switch (a.N) {
    case 16: return launch_pfb_n16(a, s);
    case 32: return launch_pfb_n32(a, s);
    case 64: return launch_pfb_n64(a, s);
    case 128: return launch_pfb_n128(a, s);
    case 256: return launch_pfb_n256(a, s);
    case 512: return launch_pfb_n512(a, s);
    case 1024: return launch_pfb_n1024(a, s);
    case 2048: return launch_pfb_n2048(a, s);
    case 4096: return launch_pfb_n4096(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rfk
