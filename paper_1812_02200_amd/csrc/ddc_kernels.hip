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
// The oscillator is an exact 64-bit integer accumulator.  Its 16-bit table
// index i = phi >> 48 splits into a quadrant g = i >> 14 and an offset
// r = i mod 2^14, and Tab[i] = (cos, sin)(2 pi i / 2^16) = (j)^g P[r] with
// the quarter-wave pair P[r] = (q[2^14 - r], q[r]), q[r] = fp32(sin(pi r/2^15)).
// So conj(Tab[i]) = (-j)^g conj(P[r]), and the quadrant turn is moved onto
// the input: LDS holds the four copies U_g[j] = (-j)^g u[j] (exact sign and
// swap operations), and each sample costs one (cos, sin) pair read from a
// 128 KiB table in LDS, one read of the quadrant's copy, and four FMAs.  The
// products are the same FP32 products as with the full 2^16-entry table.
//
// Chirped tones (Sec. III.C, Eq. 1) make the phase quadratic in the sample
// index, phi[m] = phi0 + m inc + K m(m-1)/2 (mod 2^64): the oscillator becomes
// a second-order accumulator (phase += rate, rate += K), started for each
// output window from the closed form.  Everything else is unchanged.
//
// Each work-group owns a contiguous range of outputs of one tone chunk, so a
// tone's consecutive outputs are written by one work-group (whole cache
// sectors reach HBM, not 8-byte fragments from different L2 slices).
#include "fft_device.hpp"
#include "rf_internal.hpp"

namespace rfk {

constexpr int kUChunk = 1024;                    // taps per LDS pass
constexpr int kPairs = kSinTabLen / 2;           // 2^14 (cos, sin) pairs
constexpr int kDdcLds = 4 * kUChunk + kPairs;    // float2 entries: 160 KiB

__device__ __forceinline__ uint32_t dvload(const VStream &vs, int64_t v)
{
    return v < vs.H ? gptr(vs.hist)[v] : gptr(vs.in)[v - vs.H];
}

// m(m-1)/2 mod 2^64, exactly (the even factor is halved first).
__device__ __forceinline__ uint64_t tri64(uint64_t m)
{
    return (m & 1) ? m * ((m - 1) >> 1) : (m >> 1) * (m - 1);
}

// One work unit: output o of tone chunk tc (tones tc*WG .. tc*WG+WG-1); the
// thread's tone's value is returned.  `lds` holds the four rotated input
// copies (first 4*kUChunk entries) and the pair table (loaded by the caller).
// Contains two barriers per tap chunk; every thread of the work-group must
// call it.
template <int WG, bool CHIRP>
__device__ __forceinline__ float2 ddc_unit(const DdcLaunch &a, int tc, int64_t o, float2 *lds)
{
    const int tid = threadIdx.x;
    const VStream &vs = a.vs;
    const int T = a.T;
    const int64_t v0 = o * a.D;
    const int t = tc * WG + tid;
    const bool live = t < a.ntones;
    uint64_t inc = 0, ph = 0, K = 0;
    if (live) {
        inc = gptr(a.inc)[t];
        const uint64_t m0 = a.base_abs + (uint64_t)v0;
        ph = gptr(a.phi0)[t] + m0 * inc;
        if constexpr (CHIRP) {
            K = gptr(a.chirp)[t];
            ph += K * tri64(m0);
            inc += K * m0;      // the phase step from sample m0 to m0+1
        }
    }
    // four interleaved partial sums (j mod 4): independent FMA chains
    float ar[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
    const char *ub = reinterpret_cast<const char *>(lds);
    const char *pt = reinterpret_cast<const char *>(lds + 4 * kUChunk);
    for (int c0 = 0; c0 < T; c0 += kUChunk) {
        const int len = min(kUChunk, T - c0);
        __syncthreads();  // previous readers are done with the copies (and the table is loaded)
        for (int j = tid; j < len; j += WG) {
            const uint32_t w = dvload(vs, v0 + c0 + j);
            const float h = gptr(a.wrev)[c0 + j];
            const float ux = h * (float)(int16_t)(w & 0xffffu), uy = h * (float)(int16_t)(w >> 16);
            float4 *d = reinterpret_cast<float4 *>(lds + 4 * j);
            d[0] = make_float4(ux, uy, uy, -ux);    // U_0 = u, U_1 = -j u
            d[1] = make_float4(-ux, -uy, -uy, ux);  // U_2 = -u, U_3 = j u
        }
        __syncthreads();
        if (live) {
            auto mac = [&](int q, uint64_t phk, uint32_t jb, int k) {
                const uint32_t hi = (uint32_t)(phk >> 32);
                const float2 p = *reinterpret_cast<const float2 *>(pt + ((hi >> 13) & 0x1fff8u));
                // quadrant copy address as one shift-and-add (the empty asm stops
                // the shift pair being rewritten as shift + mask + add)
                uint32_t g = hi >> 30;
                asm("" : "+v"(g));
                const uint32_t ua = (g << 3) + jb;
                const float2 uu = *reinterpret_cast<const float2 *>(ub + ua + 32 * k);
                // U_g * conj(cos + j sin)
                ar[q] = __builtin_fmaf(uu.x, p.x, ar[q]);
                ar[q] = __builtin_fmaf(uu.y, p.y, ar[q]);
                ai[q] = __builtin_fmaf(uu.y, p.x, ai[q]);
                ai[q] = __builtin_fmaf(-uu.x, p.y, ai[q]);
            };
            const int len8 = len & ~7;
            for (int j = 0; j < len8; j += 8) {
                // one phase chain: keep the compiler from splitting it into
                // eight strided accumulators (seven extra 64-bit adds)
                asm volatile("" : "+v"(ph), "+v"(inc));
                uint64_t p = ph;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    mac(k & 3, p, 32u * (uint32_t)j, k);
                    p += inc;
                    if constexpr (CHIRP) inc += K;
                }
                ph = p;
            }
            for (int j = len8; j < len; ++j) {
                mac(j & 3, ph, 32u * (uint32_t)j, 0);
                ph += inc;
                if constexpr (CHIRP) inc += K;
            }
        }
    }
    return make_float2((ar[0] + ar[1]) + (ar[2] + ar[3]), (ai[0] + ai[1]) + (ai[2] + ai[3]));
}

// Up to kRun consecutive outputs o .. o+cnt-1 of tone chunk tc, kept in
// registers and stored together: a tone's row segment leaves as back-to-back
// stores, 16 complex values = one whole 128-byte line when the row is aligned,
// so lines are complete before they are written back (one 8-byte store per
// output would reach HBM as partial-line writes).
constexpr int kRun = 16;
template <int WG, bool CHIRP>
__device__ __forceinline__ void ddc_run(const DdcLaunch &a, int tc, int64_t o, int cnt, float2 *lds)
{
    float2 res[kRun];
#pragma unroll
    for (int r = 0; r < kRun; ++r)
        if (r < cnt) res[r] = ddc_unit<WG, CHIRP>(a, tc, o + r, lds);
    const int t = tc * WG + (int)threadIdx.x;
    if (t < a.ntones) {
        typedef float v2 __attribute__((ext_vector_type(2)));
        RF_GLOBAL v2 *dst = reinterpret_cast<RF_GLOBAL v2 *>(gptr(a.out)) + (t * a.ld + o);
#pragma unroll
        for (int r = 0; r < kRun; ++r)
            if (r < cnt) dst[r] = v2{res[r].x, res[r].y};
    }
}

// End-of-call duties spread over `G` logical work-groups: the phase read-back
// (first work-group) and the retained history for the next call.
template <int WG>
__device__ __forceinline__ void ddc_tail(const DdcLaunch &a, int lwg, int G)
{
    const int tid = threadIdx.x;
    if (lwg == 0)
        for (int t = tid; t < a.ntones; t += WG)
            gptr(a.phase_out)[t] = gptr(a.phi0)[t] + a.phase_at * gptr(a.inc)[t] + (a.chirp ? gptr(a.chirp)[t] * tri64(a.phase_at) : 0);
    for (int64_t i = (int64_t)lwg * WG + tid; i < a.keep_len; i += (int64_t)G * WG)
        gptr(a.hist_out)[i] = dvload(a.vs, a.keep_from + i);
}

template <int WG>
__device__ __forceinline__ void load_table(const float *src, float2 *lds)
{
    typedef float v4 __attribute__((ext_vector_type(4)));
    const RF_GLOBAL v4 *s4 = reinterpret_cast<const RF_GLOBAL v4 *>(gptr(src));
    v4 *d4 = reinterpret_cast<v4 *>(lds + 4 * kUChunk);
    for (int i = threadIdx.x; i < kSinTabLen / 4; i += WG) d4[i] = s4[i];
}

// Work-group b of G takes units [b W / G, (b+1) W / G) of the W = TC * nout
// (tone chunk, output) units, outputs fastest.
template <int WG, bool CHIRP>
__global__ void __launch_bounds__(WG) ddc_bank(DdcLaunch a)
{
    __shared__ float2 lds[kDdcLds];
    load_table<WG>(a.sintab, lds);
    const int TC = (a.ntones + WG - 1) / WG;
    const int64_t W = (int64_t)TC * a.nout;
    const int64_t b = W * blockIdx.x / gridDim.x, e = W * (blockIdx.x + 1) / gridDim.x;
    for (int64_t it = b; it < e;) {
        const int tc = (int)(it / a.nout);
        const int64_t o = it - (int64_t)tc * a.nout;
        const int cnt = (int)min((int64_t)kRun, min(e - it, a.nout - o));
        ddc_run<WG, CHIRP>(a, tc, o, cnt, lds);
        it += cnt;
    }
    ddc_tail<WG>(a, blockIdx.x, gridDim.x);
}

// Grouped launch over the banks of many streams: the units of a call are its
// (tone chunk, output) pairs, outputs fastest, then one tail unit; an item
// holds a contiguous range of a call's units (all of them, or a chunk of a
// long call spread over several launches); work-group b of G takes the
// contiguous units [b W / G, (b+1) W / G) of the whole list.
// The table is the same for every bank and is loaded once per work-group.
// Grouped banks have linear oscillators (the serving path has no chirps).
template <int WG>
__global__ void __launch_bounds__(WG) ddc_group(const GroupHeader *hdr, const DdcItem *items)
{
    __shared__ float2 lds[kDdcLds];
    const int nitems = hdr->count;
    const int64_t total = hdr->total;
    if (nitems <= 0) return;
    const int64_t b = total * blockIdx.x / gridDim.x, e = total * (blockIdx.x + 1) / gridDim.x;
    if (b >= e) return;
    load_table<WG>(items[0].a.sintab, lds);
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].unit_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    for (int64_t w = b; w < e;) {
        while (lo + 1 < nitems && items[lo + 1].unit_begin <= w) ++lo;
        const DdcItem &it = items[lo];
        const int64_t k = w - it.unit_begin + it.unit_off;
        const int TC = (it.a.ntones + WG - 1) / WG;
        const int64_t nunits = (int64_t)TC * it.a.nout;
        if (k < nunits) {
            const int tc = (int)(k / it.a.nout);
            const int64_t o = k - (int64_t)tc * it.a.nout;
            const int64_t lim = min(e, it.unit_begin + it.units) - w;   // this work-group's and this item's end
            const int cnt = (int)min((int64_t)kRun, min(lim, it.a.nout - o));
            ddc_run<WG, false>(it.a, tc, o, cnt, lds);
            w += cnt;
        } else {
            ddc_tail<WG>(it.a, 0, 1);
            ++w;
        }
    }
}

int ddc_group_wg(int ntones)
{
    return ntones <= 64 ? 64 : ntones <= 128 ? 128 : ntones <= 256 ? 256 : ntones <= 512 ? 512 : 1024;
}

int64_t ddc_group_units(const DdcLaunch &a)
{
    const int wg = ddc_group_wg(a.ntones);
    const int TC = (a.ntones + wg - 1) / wg;
    return (int64_t)TC * a.nout + 1;
}

const void *ddc_group_kernel(int wg)
{
    switch (wg) {
    case 64: return reinterpret_cast<const void *>(&ddc_group<64>);
    case 128: return reinterpret_cast<const void *>(&ddc_group<128>);
    case 256: return reinterpret_cast<const void *>(&ddc_group<256>);
    case 512: return reinterpret_cast<const void *>(&ddc_group<512>);
    case 1024: return reinterpret_cast<const void *>(&ddc_group<1024>);
    default: return nullptr;
    }
}

hipError_t launch_ddc_group(int wg, const GroupHeader *hdr, const DdcItem *items, int grid, hipStream_t s)
{
    if (grid < 1) return hipErrorInvalidValue;
    switch (wg) {
    case 64: hipLaunchKernelGGL(ddc_group<64>, dim3((unsigned)grid), dim3(64), 0, s, hdr, items); break;
    case 128: hipLaunchKernelGGL(ddc_group<128>, dim3((unsigned)grid), dim3(128), 0, s, hdr, items); break;
    case 256: hipLaunchKernelGGL(ddc_group<256>, dim3((unsigned)grid), dim3(256), 0, s, hdr, items); break;
    case 512: hipLaunchKernelGGL(ddc_group<512>, dim3((unsigned)grid), dim3(512), 0, s, hdr, items); break;
    case 1024: hipLaunchKernelGGL(ddc_group<1024>, dim3((unsigned)grid), dim3(1024), 0, s, hdr, items); break;
    default: return hipErrorInvalidValue;
    }
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
    if (a.chirp)
        hipLaunchKernelGGL((ddc_bank<WG, true>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((ddc_bank<WG, false>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ddc(const DdcLaunch &a, hipStream_t s)
{
    if (a.T < 1 || a.T > 4096 || a.D < 1 || a.ntones < 1) return hipErrorInvalidValue;
    switch (ddc_group_wg(a.ntones)) {
    case 64: return launch_wg<64>(a, s);
    case 128: return launch_wg<128>(a, s);
    case 256: return launch_wg<256>(a, s);
    case 512: return launch_wg<512>(a, s);
    default: return launch_wg<1024>(a, s);
    }
}

}  // namespace rfk
