// ddc_kernels.hip -- direct-demodulation bank for gfx950.
//
// Paper Sec. III.B demodulates the raw stream against a set of tones, then
// low-passes and decimates.  For tone t and output n:
//     y_t[n] = sum_{k<T} h[k] x[m] conj(Tab[phi_t[m] >> 48]),  m = nD + T-1-k,
//     phi_t[m] = phi0_t + m inc_t (mod 2^64).
// Writing j = T-1-k and u_n[j] = h[T-1-j] x[nD + j], the tap-weighted input
// u_n is the same for every tone, so a work-group builds it once in LDS and
// every lane (one tone each) runs a single complex multiply-accumulate per
// sample against its own oscillator:
//     y_t[n] = sum_j u_n[j] conj(c_t[nD + j]).
// The oscillator is an exact 64-bit integer accumulator.  Its table lookup
// uses a half-wave sine table in LDS (2^15 FP32 values, 128 KiB):
//     sin(2 pi i/2^16) = +-S[i mod 2^15]   (sign = bit 15 of i),
//     cos(2 pi i/2^16) = sin(2 pi (i + 2^14)/2^16),
// which is bit-identical to the full 2^16-entry table because every entry is
// the same quarter-wave value q[j] = fp32(sin(pi j/2^15)) with a sign.
// The input is read from HBM once per output for all tones of a tile.
#include "fft_device.hpp"
#include "rf_internal.hpp"

namespace rfk {

__device__ __forceinline__ uint32_t dvload(const VStream &vs, int64_t v)
{
    return v < vs.H ? vs.hist[v] : vs.in[v - vs.H];
}

__device__ __forceinline__ float with_sign_of(uint32_t signsrc, float mag)
{
    // mag >= 0: OR in bit 31 of signsrc
    return __uint_as_float((signsrc & 0x80000000u) | __float_as_uint(mag));
}

// One work unit: output o of tone chunk tc (tones tc*WG .. tc*WG+WG-1).
// `u` is the work-group's LDS buffer for the tap-weighted input, `stab` the
// half-wave sine table already in LDS.  Contains two barriers; every thread of
// the work-group must call it.
template <int WG>
__device__ __forceinline__ void ddc_unit(const DdcLaunch &a, int tc, int64_t o, const float *stab, cf *u)
{
    const int tid = threadIdx.x;
    const VStream &vs = a.vs;
    const int T = a.T;
    __syncthreads();  // previous unit's readers are done with u (and the table is loaded)
    const int64_t v0 = o * a.D;
    for (int j = tid; j < T; j += WG) {
        const uint32_t w = dvload(vs, v0 + j);
        const cf x = {(float)(int16_t)(w & 0xffffu), (float)(int16_t)(w >> 16)};
        const float h = a.wrev[j];
        u[j] = {h * x.x, h * x.y};
    }
    __syncthreads();
    const int t = tc * WG + tid;
    if (t < a.ntones) {
        const uint64_t inc = a.inc[t];
        uint64_t ph = a.phi0[t] + (a.base_abs + (uint64_t)v0) * inc;
        // four interleaved partial sums (j mod 4): independent FMA chains
        float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
        auto mac = [&](int q, int j) {
            const uint32_t hi = (uint32_t)(ph >> 32);
            const uint32_t hc = hi + 0x40000000u;  // +quarter turn: cos = sin(. + pi/2)
            const float s = with_sign_of(hi, stab[(hi >> 16) & 0x7fffu]);
            const float c = with_sign_of(hc, stab[(hc >> 16) & 0x7fffu]);
            const cf uu = u[j];
            // u * conj(c + i s)
            ar[q] = __builtin_fmaf(uu.x, c, ar[q]);
            ar[q] = __builtin_fmaf(uu.y, s, ar[q]);
            ai[q] = __builtin_fmaf(uu.y, c, ai[q]);
            ai[q] = __builtin_fmaf(-uu.x, s, ai[q]);
            ph += inc;
        };
        const int T4 = T & ~3;
#pragma unroll 2
        for (int j = 0; j < T4; j += 4) {
            mac(0, j);
            mac(1, j + 1);
            mac(2, j + 2);
            mac(3, j + 3);
        }
        for (int j = T4; j < T; ++j) mac(j & 3, j);
        float *dst = a.out + 2 * ((int64_t)t * a.ld + o);
        dst[0] = (ar[0] + ar[1]) + (ar[2] + ar[3]);
        dst[1] = (ai[0] + ai[1]) + (ai[2] + ai[3]);
    }
}

// End-of-call duties spread over `G` logical work-groups: the phase read-back
// (first work-group) and the retained history for the next call.
template <int WG>
__device__ __forceinline__ void ddc_tail(const DdcLaunch &a, int lwg, int G)
{
    const int tid = threadIdx.x;
    if (lwg == 0)
        for (int t = tid; t < a.ntones; t += WG) a.phase_out[t] = a.phi0[t] + a.phase_at * a.inc[t];
    for (int64_t i = (int64_t)lwg * WG + tid; i < a.keep_len; i += (int64_t)G * WG)
        a.hist_out[i] = dvload(a.vs, a.keep_from + i);
}

template <int WG>
__device__ __forceinline__ void load_table(const float *src, float *stab)
{
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    float4 *d4 = reinterpret_cast<float4 *>(stab);
    for (int i = threadIdx.x; i < kSinTabLen / 4; i += WG) d4[i] = s4[i];
}

template <int WG>
__global__ void __launch_bounds__(WG) ddc_bank(DdcLaunch a)
{
    __shared__ float stab[kSinTabLen];
    __shared__ cf u[4096];
    load_table<WG>(a.sintab, stab);
    const int TC = (a.ntones + WG - 1) / WG;
    const int64_t nitems = (int64_t)TC * a.nout;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x)
        ddc_unit<WG>(a, (int)(it % TC), it / TC, stab, u);
    ddc_tail<WG>(a, blockIdx.x, gridDim.x);
}

// Grouped launch over the banks of many streams: work units are (tone chunk,
// output) pairs of every item plus one tail unit per item; work-groups stride
// over all of them.  The sine table is the same for every bank and is loaded
// once per work-group.
__global__ void __launch_bounds__(kDdcGroupWG) ddc_group(const GroupHeader *hdr, const DdcItem *items)
{
    constexpr int WG = kDdcGroupWG;
    __shared__ float stab[kSinTabLen];
    __shared__ cf u[4096];
    const int nitems = hdr->count;
    const int64_t total = hdr->total;
    if (nitems <= 0 || (int64_t)blockIdx.x >= total) return;
    load_table<WG>(items[0].a.sintab, stab);
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = nitems - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].unit_begin <= w) lo = mid;
            else hi = mid - 1;
        }
        const DdcItem &it = items[lo];
        const int64_t k = w - it.unit_begin;
        const int TC = (it.a.ntones + WG - 1) / WG;
        const int64_t nunits = (int64_t)TC * it.a.nout;
        if (k < nunits) {
            ddc_unit<WG>(it.a, (int)(k % TC), k / TC, stab, u);
        } else {
            __syncthreads();
            ddc_tail<WG>(it.a, 0, 1);
        }
    }
}

int64_t ddc_group_units(const DdcLaunch &a)
{
    const int TC = (a.ntones + kDdcGroupWG - 1) / kDdcGroupWG;
    return (int64_t)TC * a.nout + 1;
}

hipError_t launch_ddc_group(const GroupHeader *hdr, const DdcItem *items, int grid, hipStream_t s)
{
    if (grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(ddc_group, dim3((unsigned)grid), dim3(kDdcGroupWG), 0, s, hdr, items);
    return hipGetLastError();
}

int ddc_default_grid(int ntones, int64_t nout)
{
    (void)ntones;
    (void)nout;
    return 256;
}

template <int WG>
static hipError_t launch_wg(const DdcLaunch &a, hipStream_t s)
{
    int grid = a.grid > 0 ? a.grid : 256;
    hipLaunchKernelGGL((ddc_bank<WG>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ddc(const DdcLaunch &a, hipStream_t s)
{
    if (a.T < 1 || a.T > 4096 || a.D < 1 || a.ntones < 1) return hipErrorInvalidValue;
    if (a.ntones <= 64) return launch_wg<64>(a, s);
    if (a.ntones <= 128) return launch_wg<128>(a, s);
    if (a.ntones <= 256) return launch_wg<256>(a, s);
    if (a.ntones <= 512) return launch_wg<512>(a, s);
    return launch_wg<1024>(a, s);
}

}  // namespace rfk
