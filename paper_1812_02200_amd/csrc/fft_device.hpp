// fft_device.hpp -- register-level DFT building blocks for the gfx950 kernels.
//
// Forward DFTs, X[k] = sum_n x[n] exp(-2 pi i k n / R), results in natural
// order, for R in {2, 4, 8, 16}.  R = 8 and R = 16 are split as R = A * B
// (n = B*n1 + n2, k = k1 + A*k2):
//     X[k1 + A k2] = sum_{n2} W_B^{n2 k2} W_R^{n2 k1} sum_{n1} x[B n1 + n2] W_A^{n1 k1}
// i.e. B DFTs of size A on stride-B inputs, twiddles W_R^{n2 k1}, then A DFTs of
// size B.  Constant twiddles are written out so the compiler sees the trivial
// ones (1, -i, -1) as data moves.
#pragma once
#include <hip/hip_runtime.h>

namespace rfk {

struct alignas(8) cf {
    float x, y;
};

__device__ __forceinline__ cf cadd(cf a, cf b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cf csub(cf a, cf b) { return {a.x - b.x, a.y - b.y}; }
// a * b
__device__ __forceinline__ cf cmul(cf a, cf b)
{
    return {__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x)};
}
// a * (-i)
__device__ __forceinline__ cf mul_mi(cf a) { return {a.y, -a.x}; }

// cos(pi/8), sin(pi/8), sqrt(1/2) rounded to FP32
constexpr float kC1 = 0.92387953251128675613f;
constexpr float kS1 = 0.38268343236508977173f;
constexpr float kR2 = 0.70710678118654752440f;

// v * W16^E, W16 = exp(-2 pi i / 16), for the exponents an R=16 or R=8 split uses.
template <int E>
__device__ __forceinline__ cf tw16(cf v)
{
    constexpr int e = E & 15;
    if constexpr (e == 0) {
        return v;
    } else if constexpr (e == 1) {  // (c1, -s1)
        return {__builtin_fmaf(v.x, kC1, v.y * kS1), __builtin_fmaf(v.y, kC1, -v.x * kS1)};
    } else if constexpr (e == 2) {  // (r, -r)
        return {(v.x + v.y) * kR2, (v.y - v.x) * kR2};
    } else if constexpr (e == 3) {  // (s1, -c1)
        return {__builtin_fmaf(v.x, kS1, v.y * kC1), __builtin_fmaf(v.y, kS1, -v.x * kC1)};
    } else if constexpr (e == 4) {  // -i
        return {v.y, -v.x};
    } else if constexpr (e == 6) {  // (-r, -r)
        return {(v.y - v.x) * kR2, -(v.x + v.y) * kR2};
    } else if constexpr (e == 9) {  // (-c1, s1)
        return {-__builtin_fmaf(v.x, kC1, v.y * kS1), __builtin_fmaf(v.x, kS1, -v.y * kC1)};
    } else {
        static_assert(e == 0, "twiddle exponent not used by the R=8/16 splits");
        return v;
    }
}

__device__ __forceinline__ void dft2(cf &a, cf &b)
{
    cf t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

// In-place DFT4 of (a, b, c, d) = x[0..3].
__device__ __forceinline__ void dft4(cf &x0, cf &x1, cf &x2, cf &x3)
{
    cf a0 = cadd(x0, x2), a1 = csub(x0, x2);
    cf a2 = cadd(x1, x3), a3 = csub(x1, x3);
    x0 = cadd(a0, a2);
    x2 = csub(a0, a2);
    x1 = cadd(a1, mul_mi(a3));  // a1 - i a3
    x3 = csub(a1, mul_mi(a3));  // a1 + i a3
}

template <int R>
__device__ __forceinline__ void dft(cf *v);

template <>
__device__ __forceinline__ void dft<2>(cf *v)
{
    dft2(v[0], v[1]);
}

template <>
__device__ __forceinline__ void dft<4>(cf *v)
{
    dft4(v[0], v[1], v[2], v[3]);
}

// R = 8 = A*B with A = 4, B = 2.
template <>
__device__ __forceinline__ void dft<8>(cf *v)
{
    cf y[2][4];
#pragma unroll
    for (int n2 = 0; n2 < 2; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[2 * n1 + n2];
        dft4(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
    }
    // W8^{n2 k1} = W16^{2 n2 k1}
    y[1][1] = tw16<2>(y[1][1]);
    y[1][2] = tw16<4>(y[1][2]);
    y[1][3] = tw16<6>(y[1][3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cf a = y[0][k1], b = y[1][k1];
        dft2(a, b);
        v[k1] = a;
        v[k1 + 4] = b;
    }
}

// R = 16 = 4*4.
template <>
__device__ __forceinline__ void dft<16>(cf *v)
{
    cf y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[4 * n1 + n2];
        dft4(y[n2][0], y[n2][1], y[n2][2], y[n2][3]);
    }
    y[1][1] = tw16<1>(y[1][1]);
    y[1][2] = tw16<2>(y[1][2]);
    y[1][3] = tw16<3>(y[1][3]);
    y[2][1] = tw16<2>(y[2][1]);
    y[2][2] = tw16<4>(y[2][2]);
    y[2][3] = tw16<6>(y[2][3]);
    y[3][1] = tw16<3>(y[3][1]);
    y[3][2] = tw16<6>(y[3][2]);
    y[3][3] = tw16<9>(y[3][3]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        dft4(y[0][k1], y[1][k1], y[2][k1], y[3][k1]);
        v[k1] = y[0][k1];
        v[k1 + 4] = y[1][k1];
        v[k1 + 8] = y[2][k1];
        v[k1 + 12] = y[3][k1];
    }
}

}  // namespace rfk
