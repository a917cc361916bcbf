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

__global__ void __launch_bounds__(kFoldWG) large_fold(PfbLaunch a, cf *v)
{
    const int64_t N = a.N;
    const int M = a.M;
    const int64_t n = (int64_t)blockIdx.x * kFoldWG + threadIdx.x;
    const int64_t p0 = (int64_t)blockIdx.y * kFoldFrames;
    const VStream vs = a.vs;
    if (n < N) {
        float h[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) h[m] = m < M ? a.taps[m * N + n] : 0.f;
        const int64_t p1 = min(p0 + kFoldFrames, a.F);
        for (int64_t p = p0; p < p1; ++p) {
            cf s = {0.f, 0.f};
#pragma unroll
            for (int m = 0; m < 16; ++m) {
                if (m < M) {
                    const int64_t vi = (p + m) * N + n;
                    const uint32_t w = vi < vs.H ? vs.hist[vi] : vs.in[vi - vs.H];
                    const float xr = (float)(int16_t)(w & 0xffffu), xi = (float)(int16_t)(w >> 16);
                    s.x = __builtin_fmaf(h[m], xr, s.x);
                    s.y = __builtin_fmaf(h[m], xi, s.y);
                }
            }
            v[p * N + n] = s;
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

constexpr int kStepWG = 256;

// One radix-R Stockham pass over TB transforms of length L (row stride Lp)
// from A to B: butterfly j of span ns reads A[j + r L/R], applies
// W_{ns R}^{k r} (k = j mod ns, = W_L^{k r tstride}) and writes B[(j/ns) ns R + k + r ns].
template <int R>
__device__ __forceinline__ void stock_pass(const cf *A, cf *B, int Lp, int TB, int nb, int ns, int tstride,
                                           const cf *__restrict__ tw, int tid)
{
    for (int idx = tid; idx < TB * nb; idx += kStepWG) {
        const int t = idx / nb, j = idx - t * nb;
        const int k = j % ns;
        cf v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = A[t * Lp + j + r * nb];
        if (ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[k * r * tstride]);
        }
        dft_r<R>(v);
        const int o = (j / ns) * ns * R + k;
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
    const int tid = threadIdx.x;
    const int64_t T0 = (int64_t)blockIdx.x * TB;
    const int nload = TB * L;
    // load
    for (int idx = tid; idx < nload; idx += kStepWG) {
        int t, i;
        if (d.in_es == 1) { t = idx / L; i = idx - t * L; }
        else { i = idx / TB; t = idx - i * TB; }
        const int64_t T = T0 + t;
        cf x = {0.f, 0.f};
        if (T < total) {
            const int64_t f = T / d.C, c = T - f * d.C;
            x = d.src[f * N + c * d.in_cs + (int64_t)i * d.in_es];
        }
        A[t * Lp + i] = x;
    }
    __syncthreads();
    // Stockham passes
    int ns = 1;
    for (int ps = 0; ps < d.nr; ++ps) {
        const int R = d.rad[ps];
        const int nb = L / R;
        const int tstride = L / (ns * R);     // W_{ns R}^{e} = W_L^{e * L/(ns R)}
        switch (R) {
        case 2: stock_pass<2>(A, B, Lp, TB, nb, ns, tstride, d.tw, tid); break;
        case 3: stock_pass<3>(A, B, Lp, TB, nb, ns, tstride, d.tw, tid); break;
        case 4: stock_pass<4>(A, B, Lp, TB, nb, ns, tstride, d.tw, tid); break;
        case 5: stock_pass<5>(A, B, Lp, TB, nb, ns, tstride, d.tw, tid); break;
        default: stock_pass<8>(A, B, Lp, TB, nb, ns, tstride, d.tw, tid); break;
        }
        __syncthreads();
        cf *tmp = A;
        A = B;
        B = tmp;
        ns *= R;
    }
    // store (with the four-step twiddle W_N^{c k} when asked)
    for (int idx = tid; idx < nload; idx += kStepWG) {
        int t, k;
        if (d.out_es == 1) { t = idx / L; k = idx - t * L; }
        else { k = idx / TB; t = idx - k * TB; }
        const int64_t T = T0 + t;
        if (T >= total) continue;
        const int64_t f = T / d.C, c = T - f * d.C;
        cf x = A[t * Lp + k];
        if (d.thi) {
            const int64_t e = c * k;          // < N
            x = cmul(x, cmul(d.thi[e >> d.tsh], d.tlo[e & ((1ll << d.tsh) - 1)]));
        }
        d.dst[f * N + c * d.out_cs + (int64_t)k * d.out_es] = x;
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
        // the largest divisor <= 4096 whose cofactor is <= 4096 as well
        for (int64_t d = 4096; d >= 2; --d)
            if (N % d == 0 && N / d <= 4096) { n1 = d; break; }
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

static int step_tb(int L)
{
    int tb = 8192 / L;
    if (tb > 16) tb = 16;
    return tb < 1 ? 1 : tb;
}

static hipError_t launch_step(const StepDesc &d, int64_t N, int64_t total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    const int64_t grid = (total + d.TB - 1) / d.TB;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    const size_t lds = 2 * (size_t)d.TB * (d.L + 1) * sizeof(cf);
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
    if (gx > 0x7fffffff || gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(large_fold, dim3((unsigned)gx, (unsigned)gy), dim3(kFoldWG), 0, s, a, b.v);
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
