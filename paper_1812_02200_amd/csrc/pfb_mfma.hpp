// pfb_mfma.hpp -- polyphase FIR + DFT on MFMA with hi/lo split operands
// (N = 16, 32, 64, 128, 256).
//
// The folded frame v (FP32, from the same register-window FIR as the FFT path)
// is transformed through the factorisation N = 16 N2 (n = N2 n1 + n2,
// k = k1 + 16 k2):
//     Y[n2][k1] = W_N^{n2 k1} sum_{n1} v[N2 n1 + n2] W_16^{n1 k1}     (GEMM 1)
//     X[k1 + 16 k2] = sum_{n2} Y[n2][k1] W_N2^{n2 k2}                  (GEMM 2)
// Each GEMM is a real 32x32 block matrix times 64 columns of 16 complex
// values per wave and phase, on v_mfma_f32_16x16x32_{f16,bf16}: GEMM 1's
// matrix is the DFT16 on [Re | Im] and its columns are the (frame, n2) pairs;
// GEMM 2's matrix is block-diagonal with 16 / N2 copies of the DFT_N2, so a
// column holds 16 / N2 short transforms (N2 = 16: the DFT16 again; N2 = 1:
// no second GEMM).  Every wave therefore issues the same 48 MFMAs per phase
// whatever N, and every value passes both stages in the same precision.
//
// Both operands of every product are split into a high and a low part in the
// half format, x = hi + lo, and the products are accumulated in FP32 as
// hi*hi + hi*lo + lo*hi.  The dropped lo*lo term is 2^-22 of the product in
// FP16, far below FP32 resolution, but about 2^-16 in BF16 (8-bit
// significands), where it is of the order of the split's own residual; a
// runtime flag adds it (measured: +1.3 dB of channel SNR in BF16).
//
// FP16 has a largest finite value of 65504.  The taps are multiplied by 2^e
// when the handle is created (exact in FP32) with e chosen from the largest
// column sum of |h|, so that no GEMM operand can exceed 2^15 for any int16
// input; the outputs are multiplied by 2^-e (exact) when they are stored.
//
// One wave owns 64 / (N/4) lane groups (N/4 threads each, four columns per
// thread, four frames per phase): FIR, both GEMMs and the stores stay inside
// the wave, staged through the wave's own LDS region, and the spectra leave
// with consecutive lanes on consecutive values.
#pragma once
#include "pfb_kernels.hpp"

namespace rfk {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <int PREC>
struct MfmaPrec;

template <>
struct MfmaPrec<RF_PREC_F16> {
    typedef h8v vec;
    typedef _Float16 elem;
    static __device__ __forceinline__ f4v mma(vec a, vec b, f4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct MfmaPrec<RF_PREC_BF16> {
    typedef b8v vec;
    typedef __bf16 elem;
    static __device__ __forceinline__ f4v mma(vec a, vec b, f4v c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// hi = round(x), lo = round(x - hi) in the half format of PREC.
template <int PREC>
__device__ __forceinline__ void split8(const float (&x)[8], typename MfmaPrec<PREC>::vec &hi,
                                       typename MfmaPrec<PREC>::vec &lo)
{
    typedef typename MfmaPrec<PREC>::elem E;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        E h = (E)x[i];
        hi[i] = h;
        lo[i] = (E)(x[i] - (float)h);
    }
}

template <int N>
struct MfmaPlan {
    static_assert(N >= 16 && N <= 256 && (N & (N - 1)) == 0, "MFMA DFT sizes are 16..256");
    static constexpr int N2 = N / 16;     // second-stage length (1: no second GEMM)
    static constexpr int L = N / 4;       // FIR threads per lane group
    static constexpr int LGW = 64 / L;    // lane groups per wave
    static constexpr int NLG = 4 * LGW;   // lane groups per 256-thread work-group
    static constexpr int G = 16 / N2;     // short transforms per GEMM-2 column
};

// Each wave has two LDS regions of 64 columns x [Re | Im] x 17 floats (one
// float of padding per 16): GEMM 1's operands, then GEMM 2's; the finished
// spectra are staged as [frame][bin] with N + 1 complex values per frame in
// whichever region has been read out.
constexpr int kRowF = 17;
constexpr int kWaveF = 64 * 2 * kRowF;

// Offsets (floats) in the handle's constant table.
constexpr int kTabA1 = 0;         // DFT16 real block, 32 x 32
constexpr int kTabA2 = 1024;      // block-diagonal DFT_N2 real block, 32 x 32
constexpr int kTabTw = 2048;      // W_N^{n2 k1}, complex [n2][k1], N2 x 16
constexpr int kTabScale = 2048 + 2 * 256;   // 2^-e
constexpr int kTabFloats = kTabScale + 1;

template <int N, int M, int PREC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(M <= 8 ? 2 : 1))) pfb_fir_mfma(PfbLaunch a)
{
    using Q = MfmaPlan<N>;
    constexpr int L = Q::L, N2 = Q::N2, GC = Q::G;
    constexpr int W = FirState<N, M>::W;
    typedef MfmaPrec<PREC> MP;
    typedef typename MP::vec V8;

    __shared__ float lds[4][2][kWaveF];   // per wave: GEMM-1 operands, GEMM-2 operands

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int Gd = gridDim.x, bid = blockIdx.x;
    const int xq = Gd >> 3, xr = Gd & 7, xcd = bid & 7;
    const int lwg = xcd * xq + (xcd < xr ? xcd : xr) + (bid >> 3);

    const VStream vs = a.vs;
    const int64_t vlen = vs.H + vs.n;
    const int64_t F = a.F;
    const int RL = a.run_len;
    const int nph = RL >> 2;
    const bool lolo = (a.variant & 32) != 0;
    const int g = tid / L;                  // lane group in the work-group
    const int c = tid - g * L;              // FIR column base
    const int gw = g - wave * Q::LGW;       // lane group in the wave
    const int64_t f0 = ((int64_t)lwg * Q::NLG + g) * RL;

    // constant operands: lane l holds rows (l % 16) of tile t, K = 8 (l / 16) + i
    const float *tab = a.tw;
    V8 A1h[2], A1l[2], A2h_[2], A2l_[2];
    // N2 = 16: the second stage is the DFT16 again
    V8 (&A2h)[2] = N2 == 16 ? A1h : A2h_;
    V8 (&A2l)[2] = N2 == 16 ? A1l : A2l_;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        float x[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = tab[kTabA1 + (t * 16 + (lane & 15)) * 32 + 8 * (lane >> 4) + i];
        split8<PREC>(x, A1h[t], A1l[t]);
        if constexpr (N2 > 1 && N2 < 16) {
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = tab[kTabA2 + (t * 16 + (lane & 15)) * 32 + 8 * (lane >> 4) + i];
            split8<PREC>(x, A2h[t], A2l[t]);
        }
    }
    const int jl = lane >> 4;        // K block of the B operand / row block of the result
    const int cl = lane & 15;        // column within a 16-column tile
    // W_N^{n2 k1} for this lane's results: n2 = cl mod N2, k1 = 4 jl + i
    // (read from the table, a cache hit, where it is used: fewer live registers)
    const cf *twp = reinterpret_cast<const cf *>(tab + kTabTw) + (cl % N2) * 16 + 4 * jl;
    const float oscale = tab[kTabScale];

    FirState<N, M> st;
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < 4; ++k) st.hr[m][k] = a.taps[m * N + c + k * L];

    const int64_t wg_first = (int64_t)lwg * Q::NLG * RL;
    const int64_t wg_last = wg_first + (int64_t)Q::NLG * RL + M - 2;
    const bool fast = wg_first * N >= vs.H && (wg_last + 1) * N <= vlen;
#pragma unroll
    for (int i = 0; i < W; ++i) {
        uint32_t w[4];
        if (fast) {
            const uint32_t *p = vs.in + ((f0 + i) * N - vs.H) + c;
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = p[k * L];
        } else {
            load_block<N>(vs, vlen, f0 + i, c, w);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) st.xw[i][k].set(w[k]);
    }

    float *wb = lds[wave][0];
    float *wy = lds[wave][1];
    for (int ph = 0; ph < nph; ++ph) {
        const int64_t fp = f0 + 4 * ph;
        uint32_t pre[4][4];
        const bool more = (ph + 1 < nph) && (fp + 4 < F);
        if (more) {
#pragma unroll
            for (int i = 0; i < 4; ++i) load_block<N>(vs, vlen, fp + W + i, c, pre[i]);
        }
        // FIR: v[qf][n = c + L k] -> column q = (4 gw + qf) N2 + n2, row n1 (n = N2 n1 + n2)
#pragma unroll
        for (int qf = 0; qf < 4; ++qf) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                cf s = {0.f, 0.f};
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const cf x = st.xw[qf + m][k].get();
                    s.x = __builtin_fmaf(st.hr[m][k], x.x, s.x);
                    s.y = __builtin_fmaf(st.hr[m][k], x.y, s.y);
                }
                const int n = c + L * k;
                const int q = (4 * gw + qf) * N2 + (n % N2);
                wb[(2 * q) * kRowF + n / N2] = s.x;
                wb[(2 * q + 1) * kRowF + n / N2] = s.y;
            }
        }
        wave_fence();
        // GEMM 1, two 16-column tiles at a time: B[K = (comp, n1)][col = q];
        // N2 > 1: twiddle, then column c2 = fl N2 + k1 / GC of the second
        // region holds slot s = (k1 mod GC) N2 + n2; N2 = 1: X = Y, to the
        // staging area [frame][bin] in the second region
#pragma unroll
        for (int cp = 0; cp < 4; cp += 2) {
            cf tw[4];
            if constexpr (N2 > 1) {
#pragma unroll
                for (int i = 0; i < 4; ++i) tw[i] = twp[i];
            }
            V8 bh[2], bl[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                float x[8];
                const int q = 16 * (cp + u) + cl;
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = wb[(2 * q + (jl >> 1)) * kRowF + 8 * (jl & 1) + i];
                split8<PREC>(x, bh[u], bl[u]);
            }
            f4v acc[2][2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    f4v z = {0.f, 0.f, 0.f, 0.f};
                    z = MP::mma(A1h[t], bh[u], z);
                    z = MP::mma(A1h[t], bl[u], z);
                    z = MP::mma(A1l[t], bh[u], z);
                    if (lolo) z = MP::mma(A1l[t], bl[u], z);
                    acc[u][t] = z;
                }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = 16 * (cp + u) + cl;
                    if constexpr (N2 == 1) {
                        f2v *d = reinterpret_cast<f2v *>(wy) + q * (N + 1) + 4 * jl + i;
                        *d = f2v{acc[u][0][i], acc[u][1][i]};
                    } else {
                        const cf y = cmul(cf{acc[u][0][i], acc[u][1][i]}, tw[i]);
                        const int fl = q / N2, n2 = q % N2, k1 = 4 * jl + i;
                        const int c2 = fl * N2 + k1 / GC, sl = (k1 % GC) * N2 + n2;
                        wy[(2 * c2) * kRowF + sl] = y.x;
                        wy[(2 * c2 + 1) * kRowF + sl] = y.y;
                    }
                }
        }
        wave_fence();
        const float *stg = wy;   // where the finished spectra are staged
        if constexpr (N2 > 1) {
            // GEMM 2 from the second region, two tiles at a time; result row
            // r = 4 jl + i = gi N2 + k2 of column c2 is transform c2 GC + gi =
            // (frame fl, k1), bin k1 + 16 k2 -> staging [frame][bin] in the
            // first region (its GEMM-1 operands have all been read)
#pragma unroll
            for (int cp = 0; cp < 4; cp += 2) {
                V8 bh[2], bl[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    float x[8];
                    const int c2 = 16 * (cp + u) + cl;
#pragma unroll
                    for (int i = 0; i < 8; ++i) x[i] = wy[(2 * c2 + (jl >> 1)) * kRowF + 8 * (jl & 1) + i];
                    split8<PREC>(x, bh[u], bl[u]);
                }
                f4v acc[2][2];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int t = 0; t < 2; ++t) {
                        f4v z = {0.f, 0.f, 0.f, 0.f};
                        z = MP::mma(A2h[t], bh[u], z);
                        z = MP::mma(A2h[t], bl[u], z);
                        z = MP::mma(A2l[t], bh[u], z);
                        if (lolo) z = MP::mma(A2l[t], bl[u], z);
                        acc[u][t] = z;
                    }
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int c2 = 16 * (cp + u) + cl, r = 4 * jl + i;
                        const int tau = c2 * GC + r / N2;
                        const int fl = tau >> 4, bin = (tau & 15) + 16 * (r % N2);
                        f2v *d = reinterpret_cast<f2v *>(wb) + fl * (N + 1) + bin;
                        *d = f2v{acc[u][0][i], acc[u][1][i]};
                    }
            }
            stg = wb;
        }
        // the wave's lane groups' four frames each, consecutive lanes on
        // consecutive values, scaled back by 2^-e
#pragma unroll 1
        for (int j = 0; j < Q::LGW; ++j) {
            const int64_t run0 = ((int64_t)lwg * Q::NLG + wave * Q::LGW + j) * RL;
            const int64_t r1 = run0 + RL < F ? run0 + RL : F;
            const int64_t fg = run0 + 4 * ph;
            const f2v *src = reinterpret_cast<const f2v *>(stg) + 4 * j * (N + 1);
#pragma unroll
            for (int e = lane; e < 4 * N; e += 64) {
                const int qf = e / N, bin = e - qf * N;
                if (fg + qf < r1) {
                    const f2v v = src[qf * (N + 1) + bin];
                    __builtin_nontemporal_store(f2v{v.x * oscale, v.y * oscale},
                                                (f2v *)(a.out + 2 * ((fg + qf) * N + bin)));
                }
            }
        }
        wave_fence();
        if (more) shift_window<N, M>(st, pre);
    }

    for (int64_t i = (int64_t)bid * 256 + tid; i < a.keep_len; i += (int64_t)Gd * 256)
        a.hist_out[i] = vload(vs, a.keep_from + i);
}

template <int N, int M, int PREC>
hipError_t launch_mfma_nmp(const PfbLaunch &a, hipStream_t s)
{
    const int64_t runs = (a.F + a.run_len - 1) / a.run_len;
    int64_t wgs = (runs + MfmaPlan<N>::NLG - 1) / MfmaPlan<N>::NLG;
    if (wgs < 1) wgs = 1;
    if (wgs > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((pfb_fir_mfma<N, M, PREC>), dim3((unsigned)wgs), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int N, int PREC>
hipError_t launch_mfma_np(const PfbLaunch &a, hipStream_t s)
{
    switch (a.M) {
    case 1: return launch_mfma_nmp<N, 1, PREC>(a, s);
    case 2: return launch_mfma_nmp<N, 2, PREC>(a, s);
    case 3: return launch_mfma_nmp<N, 3, PREC>(a, s);
    case 4: return launch_mfma_nmp<N, 4, PREC>(a, s);
    case 5: return launch_mfma_nmp<N, 5, PREC>(a, s);
    case 6: return launch_mfma_nmp<N, 6, PREC>(a, s);
    case 7: return launch_mfma_nmp<N, 7, PREC>(a, s);
    case 8: return launch_mfma_nmp<N, 8, PREC>(a, s);
    case 9: return launch_mfma_nmp<N, 9, PREC>(a, s);
    case 10: return launch_mfma_nmp<N, 10, PREC>(a, s);
    case 11: return launch_mfma_nmp<N, 11, PREC>(a, s);
    case 12: return launch_mfma_nmp<N, 12, PREC>(a, s);
    case 13: return launch_mfma_nmp<N, 13, PREC>(a, s);
    case 14: return launch_mfma_nmp<N, 14, PREC>(a, s);
    case 15: return launch_mfma_nmp<N, 15, PREC>(a, s);
    case 16: return launch_mfma_nmp<N, 16, PREC>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int N>
hipError_t launch_mfma_n(const PfbLaunch &a, int prec, hipStream_t s)
{
    return prec == RF_PREC_BF16 ? launch_mfma_np<N, RF_PREC_BF16>(a, s) : launch_mfma_np<N, RF_PREC_F16>(a, s);
}

// Per-N entry points, each in its own translation unit.
hipError_t launch_pfb_mfma_n16(const PfbLaunch &a, int prec, hipStream_t s);
hipError_t launch_pfb_mfma_n32(const PfbLaunch &a, int prec, hipStream_t s);
hipError_t launch_pfb_mfma_n64(const PfbLaunch &a, int prec, hipStream_t s);
hipError_t launch_pfb_mfma_n128(const PfbLaunch &a, int prec, hipStream_t s);
hipError_t launch_pfb_mfma_n256(const PfbLaunch &a, int prec, hipStream_t s);

}  // namespace rfk
