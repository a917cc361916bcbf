// pfb_launch.hip -- host side of the PFB kernels: twiddle tables, default run
// length and dispatch over N.
#include <math.h>

#include "pfb_kernels.hpp"

namespace rfk {

int pfb_twiddle_count(int N)
{
    const int n = tw_offset(N, N);
    return n > 0 ? n : 1;
}

// Table of the pass with stride ns and radix R, at offset tw_offset(N, ns):
// entry [r][k] = exp(-2 pi i k r / (ns R)); for the radix-2 last pass of
// N = 4096, the factors exp(-2 pi i t / N), t < NT, then exp(-2 pi i b NT / N),
// b < N/(2 NT).  Computed in FP64, rounded to FP32.
void pfb_twiddle_fill(int N, float *tw)
{
    const double two_pi = 6.283185307179586476925286766559;
    auto put = [&](int i, long e, long period) {
        const double ang = -two_pi * (double)(e % period) / (double)period;
        tw[2 * i] = (float)cos(ang);
        tw[2 * i + 1] = (float)sin(ang);
    };
    tw[0] = 1.f;
    tw[1] = 0.f;
    for (int ns = pfb_fir_radix(N); ns < N; ns *= pass_radix(N, ns)) {
        const int R = pass_radix(N, ns), off = tw_offset(N, ns);
        if (R == 16 || N <= 2048) {
            for (int k = 0; k < ns; ++k)
                for (int r = 0; r < R; ++r) put(off + r * ns + k, (long)k * r, (long)ns * R);
        } else {
            const int nt = pfb_fft_team(N), nb = (N / R) / nt;
            for (int t = 0; t < nt; ++t) put(off + t, t, N);
            for (int b = 0; b < nb; ++b) put(off + nt + b, (long)b * nt, N);
        }
    }
}

int pfb_default_run_len(int N, int M, int64_t F)
{
    (void)M;
    // Aim for one round of work-groups at 512 threads per CU (two 256-thread
    // work-groups per CU up to N = 1024, one 512-thread work-group from
    // N = 2048), runs of 8 to 64 frames; a work-group holds max(1, 1024 / N)
    // lane groups, each walking one run.
    const int64_t nlg = N >= 1024 ? 1 : 1024 / N;
    const int64_t target = (N >= 2048 ? 256 : 512) * nlg;
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

// Pseudo-random 14-bit I/Q words for tuning buffers (a data-independent
// kernel still runs at different clocks on all-zero and on busy data).
__global__ void fill_iq_kernel(uint32_t *p, uint64_t n, uint32_t seed)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t x = (uint32_t)i * 2654435761u ^ seed;
        x ^= x >> 15;
        x *= 2246822519u;
        x ^= x >> 13;
        const uint32_t I = (x & 0x3fffu) - 0x2000u, Q = ((x >> 16) & 0x3fffu) - 0x2000u;
        p[i] = (I & 0xffffu) | (Q << 16);
    }
}

hipError_t fill_iq(uint32_t *p, uint64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_iq_kernel, dim3(1024), dim3(256), 0, s, p, n, 0x9e3779b9u);
    return hipGetLastError();
}

int64_t pfb_launch_wgs(const PfbLaunch &a)
{
    switch (a.N) {
    case 16: return pfb_wgs<16>(a);
    case 32: return pfb_wgs<32>(a);
    case 64: return pfb_wgs<64>(a);
    case 128: return pfb_wgs<128>(a);
    case 256: return pfb_wgs<256>(a);
    case 512: return pfb_wgs<512>(a);
    case 1024: return pfb_wgs<1024>(a);
    case 2048: return pfb_wgs<2048>(a);
    case 4096: return pfb_wgs<4096>(a);
    default: return 0;
    }
}

int pfb_group_wg_size(int N)
{
    switch (N) {
    case 2048: return PfbPlan<2048>::WG;
    case 4096: return PfbPlan<4096>::WG;
    default: return 256;
    }
}

const void *pfb_group_kernel(int N, int M)
{
    switch (N) {
    case 16: return pfb_group_fn_n16(M);
    case 32: return pfb_group_fn_n32(M);
    case 64: return pfb_group_fn_n64(M);
    case 128: return pfb_group_fn_n128(M);
    case 256: return pfb_group_fn_n256(M);
    case 512: return pfb_group_fn_n512(M);
    case 1024: return pfb_group_fn_n1024(M);
    case 2048: return pfb_group_fn_n2048(M);
    case 4096: return pfb_group_fn_n4096(M);
    default: return nullptr;
    }
}

hipError_t launch_pfb_group(int N, int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    if (grid < 1) return hipErrorInvalidValue;
    switch (N) {
    case 16: return launch_pfb_group_n16(M, hdr, items, grid, s);
    case 32: return launch_pfb_group_n32(M, hdr, items, grid, s);
    case 64: return launch_pfb_group_n64(M, hdr, items, grid, s);
    case 128: return launch_pfb_group_n128(M, hdr, items, grid, s);
    case 256: return launch_pfb_group_n256(M, hdr, items, grid, s);
    case 512: return launch_pfb_group_n512(M, hdr, items, grid, s);
    case 1024: return launch_pfb_group_n1024(M, hdr, items, grid, s);
    case 2048: return launch_pfb_group_n2048(M, hdr, items, grid, s);
    case 4096: return launch_pfb_group_n4096(M, hdr, items, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rfk
