// pfb_large.hip -- the PFB for large or non-power-of-two channel counts.
//
// The paper's bank also runs with N = 10^5 (Sec. III.A, Fig. 3) and mentions
// far larger spectra.  There a frame no longer fits one work-group, so the
// two stages run as separate passes over HBM:
//  1. fold: v_p[n] = sum_m h[mN+n] x[pN+mN+n], one thread per column walking
//     a chunk of frames (each input sample is read from HBM once; the M-1
//     older blocks come back from the cache), written to a scratch array;
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
// and, for W_N^e, the product of two tables W_N^{(e >> s) 2^s} W_N^{e mod 2^s}.
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
    auto ld = [&](int64_t vi) __attribute__((always_inline)) {
        const uint32_t w = vi < vs.H ? vs.hist[vi] : vs.in[vi - vs.H];
        return cf{(float)(int16_t)(w & 0xffffu), (float)(int16_t)(w >> 16)};
    };
    // frame chunks of kFoldFrames, strided over the grid's y dimension
    for (int64_t p0 = (int64_t)blockIdx.y * kFoldFrames; n < N && p0 < a.F;
         p0 += (int64_t)gridDim.y * kFoldFrames) {
        float h[M];
        cf xw[M];   // window: slot (b - p0) mod M holds block b
#pragma unroll
        for (int m = 0; m < M; ++m) h[m] = a.taps[m * N + n];
        const int64_t p1 = min(p0 + kFoldFrames, a.F);
        if (p0 < p1) {
#pragma unroll
            for (int m = 0; m < M - 1; ++m) xw[m] = ld((p0 + m) * N + n);
        }
        // frames in groups of M so that every window index is a constant
        for (int64_t pb = p0; pb < p1; pb += M) {
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const int64_t p = pb + q;
                if (p < p1) {
                    // block p + M - 1 enters the window, in the slot block p - 1 left
                    xw[(q + M - 1) % M] = ld((p + M - 1) * N + n);
                    cf s = {0.f, 0.f};
#pragma unroll
                    for (int m = 0; m < M; ++m) {
                        const cf x = xw[(q + m) % M];
                        s.x = __builtin_fmaf(h[m], x.x, s.x);
                        s.y = __builtin_fmaf(h[m], x.y, s.y);
                    }
                    v[p * N + n] = s;
                }
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

// Transform T = f*C + c (frame f, transform c of the frame) reads element i at
// src[f*N + c*in_cs + i*in_es] and writes bin k at dst[f*N + c*out_cs + k*out_es];
// a work-group takes TB consecutive transforms.
__global__ void __launch_bounds__(kStepWG) large_fft_step(StepDesc d, int64_t N, int64_t total)
{
    extern __shared__ cf sm[];
    const int L = d.L, TB = d.TB, Lp = L + 1;   // odd row stride: columns spread over banks
    cf *A = sm, *B = sm + (size_t)TB * Lp;
    cf *twl = B + (size_t)TB * Lp;             // W_L^j staged in LDS
    const int tid = threadIdx.x;
    __shared__ int64_t bin[16], bout[16], cidx[16];   // per transform: bases and column
    for (int j = tid; j < L; j += kStepWG) twl[j] = d.tw[j];
    const int64_t T0 = (int64_t)blockIdx.x * TB;
    if (tid < TB) {
        const int64_t T = T0 + tid;
        const int64_t f = T / d.C, c = T - f * d.C;
        bin[tid] = T < total ? f * N + c * d.in_cs : -1;
        bout[tid] = T < total ? f * N + c * d.out_cs : -1;
        cidx[tid] = c;
    }
    __syncthreads();
    const int nload = TB * L;
    const int lgtb = __builtin_ctz(TB);
    const float inv_l = 1.0f / (float)L;
    // load (along the contiguous direction: rows, or TB neighbouring columns),
    // eight independent loads in flight per thread before they land in LDS
    constexpr int U = 8;
    for (int base = 0; base < nload; base += U * kStepWG) {
        cf x[U];
        int slot[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * kStepWG + tid;
            slot[u] = -1;
            x[u] = cf{0.f, 0.f};
            if (idx < nload) {
                int t, i;
                if (d.in_es == 1) { t = qdiv(idx, inv_l); i = idx - t * L; }
                else { i = idx >> lgtb; t = idx & (TB - 1); }
                const int64_t b = bin[t];
                if (b >= 0) x[u] = d.src[b + (int64_t)i * d.in_es];
                slot[u] = t * Lp + i;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (slot[u] >= 0) A[slot[u]] = x[u];
    }
    __syncthreads();
    // Stockham passes
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
    for (int base = 0; base < nload; base += U * kStepWG) {
        cf x[U], w1[U], w2[U];
        int64_t dst[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * kStepWG + tid;
            dst[u] = -1;
            if (idx < nload) {
                int t, k;
                if (d.out_es == 1) { t = qdiv(idx, inv_l); k = idx - t * L; }
                else { k = idx >> lgtb; t = idx & (TB - 1); }
                const int64_t b = bout[t];
                if (b >= 0) {
                    dst[u] = b + (int64_t)k * d.out_es;
                    x[u] = A[t * Lp + k];
                    if (d.thi) {
                        const int64_t e = cidx[t] * k;    // < N
                        w1[u] = d.thi[e >> d.tsh];
                        w2[u] = d.tlo[e & ((1ll << d.tsh) - 1)];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (dst[u] < 0) continue;
            d.dst[dst[u]] = d.thi ? cmul(x[u], cmul(w1[u], w2[u])) : x[u];
        }
    }
}

// ------------------------------------------------------------------- host

static int split_radices(int L, int *rad)
{
    int n = 0;
    while (L % 8 == 0 && L > 8) { rad[n++] = 8; L /= 8; }
    while (L % 4 == 0) { rad[n++] = 4; L /= 4; }
    while (L % 2 == 0) { rad[n++] = 2; L /= 2; }
    while (L % 5 == 0) { rad[n++] = 5; L /= 5; }
    while (L % 3 == 0) { rad[n++] = 3; L /= 3; }
    if (L == 8) rad[n++] = 8, L = 1;
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
        // the most balanced split N1 * N2 (N1 <= N2 <= 4096): the column step,
        // whose loads and stores are strided, gets the shorter transforms and
        // so the most columns per work-group
        for (int64_t d = 2; d * d <= N; ++d)
            if (N % d == 0 && N / d <= 4096) n1 = d;
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

int large_tsh(int64_t N) { return N > 4096 ? 12 : 0; }

size_t large_table_floats(const LargePlan &pl)
{
    const int64_t hi = (pl.N >> large_tsh(pl.N)) + 1;
    return 2 * ((size_t)pl.N1 + (size_t)pl.N2 + (size_t)hi + (1ull << large_tsh(pl.N)));
}

void large_table_fill(const LargePlan &pl, float *t)
{
    const double two_pi = 6.283185307179586476925286766559;
    fill_wl(pl.N1, t);
    t += 2 * (size_t)pl.N1;
    fill_wl(pl.N2, t);
    t += 2 * (size_t)pl.N2;
    const int s = large_tsh(pl.N);
    const int64_t hi = (pl.N >> s) + 1;
    for (int64_t j = 0; j < hi; ++j) {      // W_N^{j 2^s}
        const double a = -two_pi * (double)((j << s) % pl.N) / (double)pl.N;
        t[2 * j] = (float)cos(a);
        t[2 * j + 1] = (float)sin(a);
    }
    t += 2 * (size_t)hi;
    for (int64_t j = 0; j < (1ll << s); ++j) {   // W_N^j
        const double a = -two_pi * (double)j / (double)pl.N;
        t[2 * j] = (float)cos(a);
        t[2 * j + 1] = (float)sin(a);
    }
}

// transforms per work-group, a power of two <= 16: two batches of TB*(L+1)
// points plus the L twiddles within 80 KiB of LDS (two work-groups per CU),
// or within 160 KiB when that would leave fewer than 4 columns per group
static int step_tb(int L)
{
    auto fit = [&](int bytes) {
        int tb = (bytes / 8 - L) / (2 * (L + 1));
        int p = 1;
        while (p * 2 <= tb && p * 2 <= 16) p *= 2;
        return tb < 1 ? 1 : p;
    };
    const int a = fit(80 * 1024);
    return a >= 4 ? a : fit(160 * 1024);
}

static hipError_t launch_step(const StepDesc &d, int64_t N, int64_t total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    const int64_t grid = (total + d.TB - 1) / d.TB;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = (2 * (size_t)d.TB * (d.L + 1) + (size_t)d.L) * sizeof(cf);
    hipLaunchKernelGGL(large_fft_step, dim3((unsigned)grid), dim3(kStepWG), lds, s, d, N, total);
    return hipGetLastError();
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
    const cf *thi = t2 + pl.N2;
    const cf *tlo = thi + ((N >> large_tsh(N)) + 1);
    cf *out = reinterpret_cast<cf *>(a.out);
    StepDesc d{};
    if (pl.N2 == 1) {
        // one step: every frame is one transform
        d.L = pl.N1;
        d.nr = pl.nr1;
        for (int i = 0; i < d.nr; ++i) d.rad[i] = pl.rad1[i];
        d.tw = t1;
        d.C = 1;
        d.TB = step_tb(d.L);
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
    d.TB = step_tb(d.L);
    d.in_cs = 1;
    d.in_es = pl.N2;
    d.out_cs = 1;
    d.out_es = pl.N2;
    d.thi = thi;
    d.tlo = tlo;
    d.tsh = large_tsh(N);
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
    d2.TB = step_tb(d2.L);
    d2.in_cs = pl.N2;
    d2.in_es = 1;
    d2.out_cs = 1;
    d2.out_es = pl.N1;
    d2.src = b.y;
    d2.dst = out;
    return launch_step(d2, N, a.F * pl.N1, s);
}

}  // namespace rfk
