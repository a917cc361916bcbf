// pfb_large.hip -- the PFB for large or non-power-of-two channel counts.
//
// The paper's bank also runs with N = 10^5 (Sec. III.A, Fig. 3) and mentions
// far larger spectra.  There a frame no longer fits one work-group, so the
// two stages run as separate passes over HBM:
//  1. fold: v_p[n] = sum_m h[mN+n] x[pN+mN+n], one thread per column and
//     chunk of frames, all of the chunk's input blocks requested at once (each
//     input sample is read from HBM about once: neighbouring chunks share M-1
//     blocks), written to a scratch array;
//  2. the N-point DFT of every frame by the four-step method, N = N1 * N2,
//     n = N2 n1 + n2, k = k1 + N1 k2:
//       Y[k1][n2] = W_N^{n2 k1} sum_{n1} v[N2 n1 + n2] W_{N1}^{n1 k1}
//       X[k1 + N1 k2] = sum_{n2} Y[k1][n2] W_{N2}^{n2 k2},
//     each step a batch of LDS-resident mixed-radix (2, 3, 4, 5, 8) Stockham
//     transforms of length <= 4096; a work-group transforms several
//     neighbouring columns (or rows) at once so that its loads and stores are
//     contiguous runs in HBM.  N <= 4096 that is not a power of two is one
//     step (N1 = N, N2 = 1).
// Twiddles are FP32 values of FP64 angles: W_L^j tables per transform length
// and, for W_N^e (e < N <= 2^24), the product of three 256-entry tables
// W_N^{(e >> 16) 2^16} W_N^{((e >> 8) mod 256) 2^8} W_N^{e mod 256}, small
// enough to live in LDS beside the transforms.
#include <math.h>
#include <stdlib.h>

#include "fft_device.hpp"
#include "rf_internal.hpp"

namespace rfk {

// ------------------------------------------------------------- butterflies

__device__ __forceinline__ void dft3(cf *v)
{
    const float c = -0.5f, s = 0.86602540378443864676f;   // cos, sin of 2 pi / 3
    const cf a = cadd(v[1], v[2]), b = csub(v[1], v[2]);
    const cf t = {v[0].x + c * a.x, v[0].y + c * a.y};
    const cf u = {s * b.x, s * b.y};
    v[0] = cadd(v[0], a);
    v[1] = cadd(t, mul_mi(u));        // t - i u
    v[2] = csub(t, mul_mi(u));
}

__device__ __forceinline__ void dft5(cf *v)
{
    const float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;   // cos 2pi/5, cos 4pi/5
    const float s1 = 0.95105651629515357212f, s2 = 0.58778525229247312917f;    // sin 2pi/5, sin 4pi/5
    const cf a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const cf a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const cf t1 = {v[0].x + c1 * a1.x + c2 * a2.x, v[0].y + c1 * a1.y + c2 * a2.y};
    const cf t2 = {v[0].x + c2 * a1.x + c1 * a2.x, v[0].y + c2 * a1.y + c1 * a2.y};
    const cf u1 = {s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y};
    const cf u2 = {s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y};
    v[0] = cadd(v[0], cadd(a1, a2));
    v[1] = cadd(t1, mul_mi(u1));      // t1 - i u1
    v[4] = csub(t1, mul_mi(u1));
    v[2] = cadd(t2, mul_mi(u2));
    v[3] = csub(t2, mul_mi(u2));
}

template <int R>
__device__ __forceinline__ void dft_r(cf *v)
{
    if constexpr (R == 3) dft3(v);
    else if constexpr (R == 5) dft5(v);
    else dft<R>(v);
}

// ------------------------------------------------------------------- fold

constexpr int kFoldWG = 256;
constexpr int kFoldFrames = 32;   // frames per thread

template <int M>
__global__ void __launch_bounds__(kFoldWG) large_fold(PfbLaunch a, cf *v)
{
    const int64_t N = a.N;
    const int64_t n = (int64_t)blockIdx.x * kFoldWG + threadIdx.x;
    const VStream vs = a.vs;
    // frame chunks of kFoldFrames, strided over the grid's y dimension; a
    // chunk's kFoldFrames + M - 1 input blocks are all requested before the
    // first is used, so each thread has that many loads in flight
    constexpr int NB = kFoldFrames + M - 1;
    for (int64_t p0 = (int64_t)blockIdx.y * kFoldFrames; n < N && p0 < a.F;
         p0 += (int64_t)gridDim.y * kFoldFrames) {
        float h[M];
#pragma unroll
        for (int m = 0; m < M; ++m) h[m] = a.taps[m * N + n];
        const int64_t p1 = min(p0 + kFoldFrames, a.F);
        const int64_t nb = p1 - p0 + M - 1;   // blocks this chunk reads
        uint32_t raw[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            raw[i] = 0;
            if (i < nb) {
                const int64_t vi = (p0 + i) * N + n;
                raw[i] = vi < vs.H ? vs.hist[vi] : vs.in[vi - vs.H];
            }
        }
        cf x[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) x[i] = cf{(float)(int16_t)(raw[i] & 0xffffu), (float)(int16_t)(raw[i] >> 16)};
#pragma unroll
        for (int q = 0; q < kFoldFrames; ++q) {
            if (p0 + q < p1) {
                cf s = {0.f, 0.f};
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    s.x = __builtin_fmaf(h[m], x[q + m].x, s.x);
                    s.y = __builtin_fmaf(h[m], x[q + m].y, s.y);
                }
                v[(p0 + q) * N + n] = s;
            }
        }
    }
    // retained history for the next call, spread over the whole grid
    const int64_t G = (int64_t)gridDim.x * gridDim.y;
    const int64_t b = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    for (int64_t i = b * kFoldWG + threadIdx.x; i < a.keep_len; i += G * kFoldWG) {
        const int64_t vi = a.keep_from + i;
        a.hist_out[i] = vi < vs.H ? vs.hist[vi] : vs.in[vi - vs.H];
    }
}

// --------------------------------------------------------- batched LDS FFT

constexpr int kStepWG = 512;

// One radix-R Stockham pass over TB transforms of length L (row stride Lp)
// from A to B: butterfly j of span ns reads A[j + r L/R], applies
// W_{ns R}^{k r} (k = j mod ns, = W_L^{k r tstride}) and writes B[(j/ns) ns R + k + r ns].
// a / b for 0 <= a < 2^20, 1 <= b <= 2^13 through the float reciprocal: the
// quotient (a + 1/2) / b is at least 1/(2b) away from an integer, far more
// than the rounding error, so truncation gives floor(a / b) exactly.
__device__ __forceinline__ int qdiv(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

template <int R>
__device__ __forceinline__ void stock_pass(const cf *A, cf *B, int Lp, int TB, int nb, int ns, int tstride,
                                           const cf *tw, int tid)
{
    const float inv_nb = 1.0f / (float)nb, inv_ns = 1.0f / (float)ns;
    for (int idx = tid; idx < TB * nb; idx += kStepWG) {
        const int t = qdiv(idx, inv_nb), j = idx - t * nb;
        const int q = qdiv(j, inv_ns), k = j - q * ns;
        cf v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = A[t * Lp + j + r * nb];
        if (ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[k * r * tstride]);
        }
        dft_r<R>(v);
        const int o = q * ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) B[t * Lp + o + r * ns] = v[r];
    }
}

// Buffer resources over a tile's two frames: accesses at offsets at or beyond
// the range are not made (loads return zero, stores are dropped), so every
// load and store below is issued unconditionally and the number of memory
// operations between a load and its use is fixed at compile time.
typedef unsigned int v2u __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));   // (whole-vector bit casts only)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const cf *p, uint32_t bytes)
{
    // the values are uniform; readfirstlane puts them in scalar registers
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const uint32_t n = __builtin_amdgcn_readfirstlane(bytes);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void *>(((uint64_t)hi << 32) | lo), (short)0,
                                             (int)n, 0x00020000);
}
constexpr int kOff = 1 << 30;   // an offset outside every range

// Transform T = f*C + c (frame f, transform c of the frame) reads element i at
// src[f*N + c*in_cs + i*in_es] and writes bin k at dst[f*N + c*out_cs + k*out_es];
// tile b is the TB consecutive transforms from b*TB.  The
// grid is persistent: a work-group walks tiles b, b + G, ...; the loads of its
// next tile are issued before the passes of the current one and land in LDS
// only after its stores have been issued (U per thread, TB*L <= U*kStepWG), so
// a tile's loads and stores overlap the neighbouring tiles' work.
template <int U>
__global__ void __launch_bounds__(kStepWG) large_fft_step(StepDesc d, int64_t N, int64_t total, int64_t ntiles)
{
    extern __shared__ cf sm[];
    const int L = d.L, TB = d.TB, Lp = L + 1;   // odd row stride: columns spread over banks
    cf *const A0 = sm, *const B0 = sm + (size_t)TB * Lp;
    cf *twl = B0 + (size_t)TB * Lp;            // W_L^j staged in LDS
    cf *t3l = twl + L;                         // the four-step tables, when used
    const int tid = threadIdx.x;
    // per transform of a tile: input and output offsets (elements, from the
    // tile's first frame) and column; two sets, for the tile being stored and
    // the tile being loaded
    __shared__ int32_t bin[2][16], bout[2][16], cidx[2][16];
    for (int j = tid; j < L; j += kStepWG) twl[j] = d.tw[j];
    if (d.t3)
        for (int j = tid; j < 768; j += kStepWG) t3l[j] = d.t3[j];
    const int nload = TB * L;
    const int lgtb = __builtin_ctz(TB);
    const float inv_l = 1.0f / (float)L;
    // a tile's transforms lie in at most TB/C + 2 frames; below 2^30 bytes for
    // every supported N (N <= 2^24 with C >= TB, or N <= 4096 C)
    const uint32_t span = (uint32_t)((TB / d.C + 2) * N * (int64_t)sizeof(cf));
    auto frame0 = [&](int64_t tile) __attribute__((always_inline)) { return tile * TB / d.C; };
    auto bases = [&](int64_t tile, int s) __attribute__((always_inline)) {
        if (tid < TB) {
            const int64_t T = tile * TB + tid;
            const int64_t f = T / d.C, c = T - f * d.C;
            const int64_t rel = (f - frame0(tile)) * N;
            bin[s][tid] = T < total ? (int32_t)(rel + c * d.in_cs) : -1;
            bout[s][tid] = T < total ? (int32_t)(rel + c * d.out_cs) : -1;
            cidx[s][tid] = (int32_t)c;
        }
    };
    // element u of this thread: idx = u*kStepWG + tid, along the contiguous
    // direction (rows, or TB neighbouring columns)
    auto slot_of = [&](int idx, int &t, int &i) __attribute__((always_inline)) {
        if (d.in_es == 1) { t = qdiv(idx, inv_l); i = idx - t * L; }
        else { i = idx >> lgtb; t = idx & (TB - 1); }
    };
    cf x[U];
    auto load = [&](int64_t tile, int s) __attribute__((always_inline)) {
        const __amdgpu_buffer_rsrc_t r =
            tile_rsrc(d.src + frame0(tile) * N, tile < ntiles ? span : 0u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = u * kStepWG + tid;
            int t = 0, i = 0, off = kOff;
            if (idx < nload) {
                slot_of(idx, t, i);
                const int b = bin[s][t];
                if (b >= 0) off = (b + i * (int)d.in_es) * (int)sizeof(cf);
            }
            const v2f w = __builtin_bit_cast(v2f, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
            x[u] = cf{w.x, w.y};
        }
    };
    auto put = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = u * kStepWG + tid;
            if (idx < nload) {
                int t, i;
                slot_of(idx, t, i);
                A0[t * Lp + i] = x[u];
            }
        }
    };

    int64_t tile = blockIdx.x;
    bases(tile, 0);
    __syncthreads();   // twiddles and the first bases
    load(tile, 0);
    put();
    for (int s = 0; tile < ntiles; tile += gridDim.x, s ^= 1) {
        const int64_t nxt = tile + gridDim.x;
        if (nxt < ntiles) bases(nxt, s ^ 1);
        __syncthreads();   // this tile in LDS, the next tile's bases visible
        load(nxt, s ^ 1);  // a zero-range resource past the last tile: no access
        // Stockham passes
        cf *A = A0, *B = B0;
        int ns = 1;
        for (int ps = 0; ps < d.nr; ++ps) {
            const int R = d.rad[ps];
            const int nb = L / R;
            const int tstride = L / (ns * R);     // W_{ns R}^{e} = W_L^{e * L/(ns R)}
            switch (R) {
            case 2: stock_pass<2>(A, B, Lp, TB, nb, ns, tstride, twl, tid); break;
            case 3: stock_pass<3>(A, B, Lp, TB, nb, ns, tstride, twl, tid); break;
            case 4: stock_pass<4>(A, B, Lp, TB, nb, ns, tstride, twl, tid); break;
            case 5: stock_pass<5>(A, B, Lp, TB, nb, ns, tstride, twl, tid); break;
            default: stock_pass<8>(A, B, Lp, TB, nb, ns, tstride, twl, tid); break;
            }
            __syncthreads();
            cf *tmp = A;
            A = B;
            B = tmp;
            ns *= R;
        }
        // store (with the four-step twiddle W_N^{c k} when asked)
        const __amdgpu_buffer_rsrc_t w = tile_rsrc(d.dst + frame0(tile) * N, span);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = u * kStepWG + tid;
            int off = kOff;
            cf y = {0.f, 0.f};
            if (idx < nload) {
                int t, k;
                if (d.out_es == 1) { t = qdiv(idx, inv_l); k = idx - t * L; }
                else { k = idx >> lgtb; t = idx & (TB - 1); }
                const int b = bout[s][t];
                if (b >= 0) {
                    off = (b + k * (int)d.out_es) * (int)sizeof(cf);
                    y = A[t * Lp + k];
                    if (d.t3) {
                        const int e = cidx[s][t] * k;    // < N <= 2^24
                        y = cmul(y, cmul(cmul(t3l[512 + (e >> 16)], t3l[256 + ((e >> 8) & 255)]),
                                         t3l[e & 255]));
                    }
                }
            }
            v2f v;
            v.x = y.x;
            v.y = y.y;
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, v), w, off, 0, 0);
        }
        __syncthreads();   // the tile buffers and this set of bases are free again
        put();             // the next tile (its loads have had the passes and stores to land)
    }
}

// ------------------------------------------------------------------- host

static int split_radices(int L, int *rad)
{
    int n = 0;
    while (L % 8 == 0) { rad[n++] = 8; L /= 8; }
    while (L % 4 == 0) { rad[n++] = 4; L /= 4; }
    while (L % 2 == 0) { rad[n++] = 2; L /= 2; }
    while (L % 5 == 0) { rad[n++] = 5; L /= 5; }
    while (L % 3 == 0) { rad[n++] = 3; L /= 3; }
    return L == 1 ? n : -1;
}

bool large_supported(int64_t N)
{
    if (N < 16 || N > (1 << 24)) return false;
    LargePlan pl;
    return large_plan(N, &pl);
}

bool large_plan(int64_t N, LargePlan *pl)
{
    int64_t r = N;
    for (int q : {2, 3, 5})
        while (r % q == 0) r /= q;
    if (r != 1) return false;
    int64_t n1 = 0, n2 = 1;
    if (N <= 4096) {
        n1 = N;
    } else {
        // N1 * N2 with N1 <= N2 <= 4096: the column step, whose loads and
        // stores are strided, gets the shorter transforms and so the most
        // columns per work-group.  Among the splits within a factor of two of
        // the balanced one, the fewest Stockham passes in all (each pass is a
        // round trip through LDS and a barrier), the most balanced on a tie;
        // else the most balanced split.
        int best = 1 << 30;
        int tmp[16];
        for (int64_t d = 2; d * d <= N; ++d) {
            if (N % d || N / d > 4096) continue;
            if (4 * d * d >= N) {
                const int p1 = split_radices((int)d, tmp), p2 = split_radices((int)(N / d), tmp);
                if (p1 > 0 && p2 > 0 && p1 + p2 <= best) {
                    best = p1 + p2;
                    n1 = d;
                }
            } else if (best == (1 << 30)) {
                n1 = d;
            }
        }
        if (!n1) return false;
        n2 = N / n1;
    }
    pl->N = N;
    pl->N1 = (int)n1;
    pl->N2 = (int)n2;
    pl->nr1 = split_radices((int)n1, pl->rad1);
    pl->nr2 = n2 > 1 ? split_radices((int)n2, pl->rad2) : 0;
    return pl->nr1 > 0 && (n2 == 1 || pl->nr2 > 0);
}

static void fill_wl(int64_t L, float *tw)   // W_L^j = exp(-2 pi i j / L), j < L
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t j = 0; j < L; ++j) {
        const double a = -two_pi * (double)j / (double)L;
        tw[2 * j] = (float)cos(a);
        tw[2 * j + 1] = (float)sin(a);
    }
}

size_t large_table_floats(const LargePlan &pl)
{
    return 2 * ((size_t)pl.N1 + (size_t)pl.N2 + 768);
}

void large_table_fill(const LargePlan &pl, float *t)
{
    const double two_pi = 6.283185307179586476925286766559;
    fill_wl(pl.N1, t);
    t += 2 * (size_t)pl.N1;
    fill_wl(pl.N2, t);
    t += 2 * (size_t)pl.N2;
    // W_N^{j}, W_N^{256 j}, W_N^{65536 j} for j < 256 (exponents reduced mod N)
    for (int lvl = 0; lvl < 3; ++lvl)
        for (int64_t j = 0; j < 256; ++j) {
            const int64_t e = (j << (8 * lvl)) % pl.N;
            const double a = -two_pi * (double)e / (double)pl.N;
            t[2 * (256 * lvl + j)] = (float)cos(a);
            t[2 * (256 * lvl + j) + 1] = (float)sin(a);
        }
}

// transforms per work-group, a power of two <= 16: two batches of TB*(L+1)
// points plus the L twiddles (and `extra` more values) within 80 KiB of LDS
// (two work-groups per CU) and at most 8 points per thread, or within 160 KiB
// and 16 points per thread when that would leave fewer than 4 columns per group
static int step_tb(int L, int extra)
{
    auto fit = [&](int bytes, int pts) {
        int tb = (bytes / 8 - L - extra) / (2 * (L + 1));
        if (tb > pts * kStepWG / L) tb = pts * kStepWG / L;
        int p = 1;
        while (p * 2 <= tb && p * 2 <= 16) p *= 2;
        return tb < 1 ? 1 : p;
    };
    const int a = fit(80 * 1024, 8);
    return a >= 4 ? a : fit(160 * 1024, 16);
}

template <int U>
static hipError_t launch_step_u(const StepDesc &d, int64_t N, int64_t total, hipStream_t s)
{
    const int64_t ntiles = (total + d.TB - 1) / d.TB;
    const size_t lds = (2 * (size_t)d.TB * (d.L + 1) + (size_t)d.L + (d.t3 ? 768 : 0)) * sizeof(cf);
    // persistent grid: the work-groups that are resident at once
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, large_fft_step<U>, kStepWG, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int64_t grid = ntiles < (int64_t)per_cu * cus ? ntiles : (int64_t)per_cu * cus;
    hipLaunchKernelGGL(large_fft_step<U>, dim3((unsigned)grid), dim3(kStepWG), lds, s, d, N, total, ntiles);
    return hipGetLastError();
}

static hipError_t launch_step(const StepDesc &d, int64_t N, int64_t total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    // the kernel addresses a tile's frames through a range below kOff bytes
    if ((int64_t)(d.TB / d.C + 2) * N * (int64_t)sizeof(cf) >= kOff) return hipErrorInvalidValue;
    const int64_t pts = (int64_t)d.TB * d.L;
    if (pts <= 8 * kStepWG) return launch_step_u<8>(d, N, total, s);
    if (pts <= 16 * kStepWG) return launch_step_u<16>(d, N, total, s);
    return hipErrorInvalidValue;
}

hipError_t launch_pfb_large(const PfbLaunch &a, const LargePlan &pl, const LargeBuffers &b, hipStream_t s)
{
    const int64_t N = a.N;
    // fold (always launched: it also moves the retained history)
    const int64_t gx = (N + kFoldWG - 1) / kFoldWG;
    int64_t gy = (a.F + kFoldFrames - 1) / kFoldFrames;
    if (gy < 1) gy = 1;
    if (gy > 65535) gy = 65535;        // the kernel strides over further chunks
    if (gx > 0x7fffffff) return hipErrorInvalidValue;
    switch (a.M) {
#define RF_FOLD_CASE(m) \
    case m: hipLaunchKernelGGL(large_fold<m>, dim3((unsigned)gx, (unsigned)gy), dim3(kFoldWG), 0, s, a, b.v); break;
        RF_FOLD_CASE(1) RF_FOLD_CASE(2) RF_FOLD_CASE(3) RF_FOLD_CASE(4) RF_FOLD_CASE(5) RF_FOLD_CASE(6)
        RF_FOLD_CASE(7) RF_FOLD_CASE(8) RF_FOLD_CASE(9) RF_FOLD_CASE(10) RF_FOLD_CASE(11) RF_FOLD_CASE(12)
        RF_FOLD_CASE(13) RF_FOLD_CASE(14) RF_FOLD_CASE(15) RF_FOLD_CASE(16)
#undef RF_FOLD_CASE
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.F == 0) return e;
    const cf *t1 = reinterpret_cast<const cf *>(b.tables);
    const cf *t2 = t1 + pl.N1;
    const cf *t3 = t2 + pl.N2;
    cf *out = reinterpret_cast<cf *>(a.out);
    StepDesc d{};
    if (pl.N2 == 1) {
        // one step: every frame is one transform
        d.L = pl.N1;
        d.nr = pl.nr1;
        for (int i = 0; i < d.nr; ++i) d.rad[i] = pl.rad1[i];
        d.tw = t1;
        d.C = 1;
        d.TB = step_tb(d.L, 0);
        d.in_cs = d.out_cs = 0;
        d.in_es = d.out_es = 1;
        d.src = b.v;
        d.dst = out;
        return launch_step(d, N, a.F, s);
    }
    // step 1: N2 column transforms of length N1 per frame, then W_N^{n2 k1}
    d.L = pl.N1;
    d.nr = pl.nr1;
    for (int i = 0; i < d.nr; ++i) d.rad[i] = pl.rad1[i];
    d.tw = t1;
    d.C = pl.N2;
    d.TB = step_tb(d.L, 768);
    d.in_cs = 1;
    d.in_es = pl.N2;
    d.out_cs = 1;
    d.out_es = pl.N2;
    d.t3 = t3;
    d.src = b.v;
    d.dst = b.y;
    e = launch_step(d, N, a.F * pl.N2, s);
    if (e != hipSuccess) return e;
    // step 2: N1 row transforms of length N2 per frame, bins k1 + N1 k2
    StepDesc d2{};
    d2.L = pl.N2;
    d2.nr = pl.nr2;
    for (int i = 0; i < d2.nr; ++i) d2.rad[i] = pl.rad2[i];
    d2.tw = t2;
    d2.C = pl.N1;
    d2.TB = step_tb(d2.L, 0);
    d2.in_cs = pl.N2;
    d2.in_es = 1;
    d2.out_cs = 1;
    d2.out_es = pl.N1;
    d2.src = b.y;
    d2.dst = out;
    return launch_step(d2, N, a.F * pl.N1, s);
}

}  // namespace rfk
