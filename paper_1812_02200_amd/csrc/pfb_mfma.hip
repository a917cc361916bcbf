// pfb_mfma.hip -- polyphase FIR + DFT on MFMA with hi/lo split operands (N = 256).
//
// The folded frame v (FP32, from the same register-window FIR as the FFT
// path) is transformed as X = v W with W the 256-point DFT matrix, computed
// through the Cooley-Tukey factorisation 256 = 16 x 16 (n = 16 n1 + n2,
// k = k1 + 16 k2):
//     Y[n2][k1] = sum_{n1} v[16 n1 + n2] W16^{n1 k1}          (GEMM 1)
//     Y[n2][k1] *= W256^{n2 k1}                                (FP32)
//     X[k1 + 16 k2] = sum_{n2} Y[n2][k1] W16^{n2 k2}          (GEMM 2)
// Each GEMM is a real 32x32 block matrix (the DFT16 on [Re | Im]) times the
// data, on v_mfma_f32_16x16x32_{f16,bf16}.  Both operands are split into a
// high and a low half-precision part, and the product is accumulated in FP32
// as hi*hi + hi*lo + lo*hi (the lo*lo term is below FP32 resolution).
// One wave owns one lane group (64 threads) and its four frames per phase:
// FIR, both GEMMs and the stores stay inside the wave.
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

// LDS layout of a folded frame for GEMM 1: [comp][n2][n1] with rows of 17
// floats (n1 fastest, one float of padding), so a lane reads 8 consecutive n1.
constexpr int kRow = 17;
constexpr int kFrameF = 2 * 16 * kRow;   // floats per frame

template <int M, int PREC>
__global__ void __launch_bounds__(256) pfb_fir_mfma256(PfbLaunch a)
{
    constexpr int N = 256;
    using P = PfbPlan<N>;          // L = 64: one lane group per wave, 4 per work-group
    constexpr int L = P::L;
    constexpr int W = FirState<N, M>::W;
    typedef MfmaPrec<PREC> MP;
    typedef typename MP::vec V8;

    // per wave: 4 frames of v, then the same space for Y
    __shared__ float vbuf[4][4 * kFrameF];

    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int G = gridDim.x, bid = blockIdx.x;
    const int xq = G >> 3, xr = G & 7, xcd = bid & 7;
    const int lwg = xcd * xq + (xcd < xr ? xcd : xr) + (bid >> 3);

    const VStream vs = a.vs;
    const int64_t vlen = vs.H + vs.n;
    const int64_t F = a.F;
    const int RL = a.run_len;
    const int nph = RL >> 2;
    const int c = lane;                                  // FIR column base (L = 64)
    const int64_t f0 = ((int64_t)lwg * P::NLG + wave) * RL;
    const int64_t f1 = (f0 + RL < F) ? f0 + RL : F;

    // DFT16 as a real 32x32 block matrix, rows = output (k, re|im), cols = input
    // (n, re|im); lane l holds rows (l%16) of tile t and k = 8(l/16)+i.
    V8 Ahi[2], Alo[2];
    {
        const float *dm = a.tw;   // 2 tiles x 16 rows x 32 k, FP32, precomputed on the host
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = dm[(t * 16 + (lane & 15)) * 32 + 8 * (lane >> 4) + i];
            split8<PREC>(x, Ahi[t], Alo[t]);
        }
    }
    // inter-stage twiddles W256^{n2 k1}: n2 = lane%16, k1 = 4(lane/16)+i
    cf tw[4];
    {
        const cf *t2 = reinterpret_cast<const cf *>(a.tw + 2 * 16 * 32);
#pragma unroll
        for (int i = 0; i < 4; ++i) tw[i] = t2[(lane & 15) * 16 + 4 * (lane >> 4) + i];
    }

    FirState<N, M> st;
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < 4; ++k) st.hr[m][k] = a.taps[m * N + c + k * L];

    const int64_t wg_first = (int64_t)lwg * P::NLG * RL;
    const int64_t wg_last = wg_first + (int64_t)P::NLG * RL + M - 2;
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

    float *vb = vbuf[wave];
    const int n2l = lane & 15;       // GEMM column (n2 in stage 1, k1 in stage 2)
    const int jl = lane >> 4;        // K block: 0,1 -> Re n in [8j, 8j+8); 2,3 -> Im
    const int comp_l = jl >> 1;
    const int kofs = 8 * (jl & 1);

    for (int ph = 0; ph < nph; ++ph) {
        const int64_t fp = f0 + 4 * ph;
        uint32_t pre[4][4];
        const bool more = (ph + 1 < nph) && (fp + 4 < F);
        if (more) {
#pragma unroll
            for (int i = 0; i < 4; ++i) load_block<N>(vs, vlen, fp + W + i, c, pre[i]);
        }
        // FIR: v[qf][c + 64k] -> LDS [qf][comp][n2][n1] with n = 16 n1 + n2
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
                const int n = c + 64 * k;
                const int n1 = n >> 4, n2 = n & 15;
                vb[qf * kFrameF + (0 * 16 + n2) * kRow + n1] = s.x;
                vb[qf * kFrameF + (1 * 16 + n2) * kRow + n1] = s.y;
            }
        }
        wave_fence();
#pragma unroll
        for (int qf = 0; qf < 4; ++qf) {
            float *fb = vb + qf * kFrameF;
            // GEMM 1: B operand = v[16 n1 + n2] for column n2 = lane%16, K rows kofs..+8
            float x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = fb[(comp_l * 16 + n2l) * kRow + kofs + i];
            V8 bh, bl;
            split8<PREC>(x, bh, bl);
            f4v acc[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                f4v z = {0.f, 0.f, 0.f, 0.f};
                z = MP::mma(Ahi[t], bh, z);
                z = MP::mma(Ahi[t], bl, z);
                z = MP::mma(Alo[t], bh, z);
                acc[t] = z;
            }
            wave_fence();
            // Y[n2 = lane%16][k1 = 4(lane/16)+i] (tile 0: Re, tile 1: Im), twiddled,
            // back to LDS as [comp][k1][n2] for GEMM 2
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const cf y = cmul(cf{acc[0][i], acc[1][i]}, tw[i]);
                const int k1 = 4 * jl + i;
                fb[(0 * 16 + k1) * kRow + n2l] = y.x;
                fb[(1 * 16 + k1) * kRow + n2l] = y.y;
            }
            wave_fence();
            // GEMM 2: B operand = Y[n2 = kofs..+8][k1 = lane%16]
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = fb[(comp_l * 16 + n2l) * kRow + kofs + i];
            split8<PREC>(x, bh, bl);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                f4v z = {0.f, 0.f, 0.f, 0.f};
                z = MP::mma(Ahi[t], bh, z);
                z = MP::mma(Ahi[t], bl, z);
                z = MP::mma(Alo[t], bh, z);
                acc[t] = z;
            }
            // X[k1 + 16 k2], k1 = lane%16, k2 = 4(lane/16)+i
            const int64_t f = fp + qf;
            if (f < f1) {
                float *o = a.out + 2 * f * (int64_t)N;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    f2v val = {acc[0][i], acc[1][i]};
                    __builtin_nontemporal_store(val, (f2v *)(o + 2 * (n2l + 16 * (4 * jl + i))));
                }
            }
        }
        wave_fence();
        if (more) shift_window<N, M>(st, pre);
    }

    for (int64_t i = (int64_t)bid * 256 + tid; i < a.keep_len; i += (int64_t)G * 256)
        a.hist_out[i] = vload(vs, a.keep_from + i);
}

// Host: constant tables for the MFMA path, laid out as the kernel reads them:
// [0, 1024) floats: DFT16 real block matrix, 2 row tiles x 16 rows x 32 columns;
// [1024, 1024 + 512) floats: W256^{n2 k1} as complex [n2][k1].
int pfb_mfma_table_floats() { return 2 * 16 * 32 + 2 * 256; }

void pfb_mfma_table_fill(float *t)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int row = 0; row < 32; ++row)
        for (int q = 0; q < 32; ++q) {
            const int k = row & 15, n = q & 15;
            const double th = two_pi * (double)((k * n) % 16) / 16.0;
            double v;
            if (row < 16)   // Re Y[k] = sum Re z cos + Im z sin
                v = (q < 16) ? cos(th) : sin(th);
            else            // Im Y[k] = sum Im z cos - Re z sin
                v = (q < 16) ? -sin(th) : cos(th);
            t[row * 32 + q] = (float)v;
        }
    float *w = t + 2 * 16 * 32;
    for (int n2 = 0; n2 < 16; ++n2)
        for (int k1 = 0; k1 < 16; ++k1) {
            const double th = -two_pi * (double)((n2 * k1) % 256) / 256.0;
            w[2 * (n2 * 16 + k1)] = (float)cos(th);
            w[2 * (n2 * 16 + k1) + 1] = (float)sin(th);
        }
}

template <int M, int PREC>
static hipError_t launch_m(const PfbLaunch &a, hipStream_t s)
{
    const int64_t runs = (a.F + a.run_len - 1) / a.run_len;
    int64_t wgs = (runs + 3) / 4;
    if (wgs < 1) wgs = 1;
    if (wgs > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((pfb_fir_mfma256<M, PREC>), dim3((unsigned)wgs), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int PREC>
static hipError_t launch_p(const PfbLaunch &a, hipStream_t s)
{
    switch (a.M) {
    case 1: return launch_m<1, PREC>(a, s);
    case 2: return launch_m<2, PREC>(a, s);
    case 3: return launch_m<3, PREC>(a, s);
    case 4: return launch_m<4, PREC>(a, s);
    case 5: return launch_m<5, PREC>(a, s);
    case 6: return launch_m<6, PREC>(a, s);
    case 7: return launch_m<7, PREC>(a, s);
    case 8: return launch_m<8, PREC>(a, s);
    case 9: return launch_m<9, PREC>(a, s);
    case 10: return launch_m<10, PREC>(a, s);
    case 11: return launch_m<11, PREC>(a, s);
    case 12: return launch_m<12, PREC>(a, s);
    case 13: return launch_m<13, PREC>(a, s);
    case 14: return launch_m<14, PREC>(a, s);
    case 15: return launch_m<15, PREC>(a, s);
    case 16: return launch_m<16, PREC>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pfb_mfma(const PfbLaunch &a, int prec, hipStream_t s)
{
    if (a.N != 256 || a.run_len <= 0 || (a.run_len & 3)) return hipErrorInvalidValue;
    return prec == RF_PREC_BF16 ? launch_p<RF_PREC_BF16>(a, s) : launch_p<RF_PREC_F16>(a, s);
}

}  // namespace rfk
