// pfb_mfma.hip -- host side of the MFMA DFT path: the handle's constant table
// (the two real block matrices, the inter-stage twiddles and the output scale),
// the tap scale exponent, and dispatch over N.
#include <math.h>

#include "pfb_mfma.hpp"

namespace rfk {

int pfb_mfma_table_floats() { return kTabFloats; }

// Largest power-of-two exponent e (within [-100, 100]) for which no GEMM
// operand can exceed 2^15 when the taps are scaled by 2^e: a folded value
// has components of at most 32768 * S (S = the largest column sum of |h|, an
// int16 input at most 32768 in magnitude) and modulus at most sqrt(2) times
// that; GEMM 2's operands are the twiddled DFT16 of 16 such values, at most
// 16 sqrt(2) 32768 S.  Returns false when no such e exists.
bool pfb_mfma_scale_exponent(const float *h, int N, int M, int *e_out)
{
    double S = 0.0;
    for (int n = 0; n < N; ++n) {
        double s = 0.0;
        for (int m = 0; m < M; ++m) s += fabs((double)h[m * N + n]);
        if (s > S) S = s;
    }
    const double bound = 32768.0 * S * (N > 16 ? 16.0 * sqrt(2.0) : 1.0);
    if (bound == 0.0) {
        *e_out = 0;
        return true;
    }
    int e = (int)floor(log2(32768.0 / bound));
    if (e > 100) e = 100;
    if (e < -100) return false;
    while (e > -100 && ldexp(bound, e) > 32768.0) --e;   // guard the floor against rounding
    *e_out = e;
    return ldexp(bound, e) <= 32768.0;
}

// [kTabA1]: DFT16 real block, rows (Re k | Im k), columns (Re n | Im n);
// [kTabA2]: the block-diagonal DFT_N2 in the same layout over slots
// s = g N2 + j (blocks g = 0 .. 16/N2 - 1; N2 = 1: unused);
// [kTabTw]: W_N^{n2 k1} as complex [n2][k1]; [kTabScale]: 2^-e.
void pfb_mfma_table_fill(int N, int scale_exp, float *t)
{
    const double two_pi = 6.283185307179586476925286766559;
    const int N2 = N / 16;
    for (int i = 0; i < kTabFloats; ++i) t[i] = 0.f;
    for (int row = 0; row < 32; ++row)
        for (int q = 0; q < 32; ++q) {
            const int k = row & 15, n = q & 15;
            // A1: Re Y[k] = sum Re z cos + Im z sin, Im Y[k] = sum Im z cos - Re z sin
            {
                const double th = two_pi * (double)((k * n) % 16) / 16.0;
                double v;
                if (row < 16) v = (q < 16) ? cos(th) : sin(th);
                else v = (q < 16) ? -sin(th) : cos(th);
                t[kTabA1 + row * 32 + q] = (float)v;
            }
            // A2: zero between different blocks, the DFT_N2 inside a block
            if (N2 > 1 && k / N2 == n / N2) {
                const int k2 = k % N2, n2 = n % N2;
                const double th = two_pi * (double)((k2 * n2) % N2) / (double)N2;
                double v;
                if (row < 16) v = (q < 16) ? cos(th) : sin(th);
                else v = (q < 16) ? -sin(th) : cos(th);
                t[kTabA2 + row * 32 + q] = (float)v;
            }
        }
    for (int n2 = 0; n2 < N2; ++n2)
        for (int k1 = 0; k1 < 16; ++k1) {
            const double th = -two_pi * (double)((n2 * k1) % N) / (double)N;
            t[kTabTw + 2 * (n2 * 16 + k1)] = (float)cos(th);
            t[kTabTw + 2 * (n2 * 16 + k1) + 1] = (float)sin(th);
        }
    t[kTabScale] = ldexpf(1.0f, -scale_exp);
}

hipError_t launch_pfb_mfma(const PfbLaunch &a, int prec, hipStream_t s)
{
    if (a.run_len <= 0 || (a.run_len & 3)) return hipErrorInvalidValue;
    switch (a.N) {
    case 16: return launch_pfb_mfma_n16(a, prec, s);
    case 32: return launch_pfb_mfma_n32(a, prec, s);
    case 64: return launch_pfb_mfma_n64(a, prec, s);
    case 128: return launch_pfb_mfma_n128(a, prec, s);
    case 256: return launch_pfb_mfma_n256(a, prec, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rfk
