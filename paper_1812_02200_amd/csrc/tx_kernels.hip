// tx_kernels.hip -- multi-tone transmit synthesis (DAC buffers) for gfx950.
//
// The readout generates its transmit buffers on the GPU (paper Sec. III),
// including chirped excitations (Sec. III.C, Eq. 1).  Tone t carries an
// oscillator state at the buffer's first sample -- phase phi_t, rate r_t
// (phase step to the next sample) and second difference K_t (0 for a fixed
// frequency) -- and an amplitude a_t in DAC counts.  Sample j is
//     v[j] = sum_t a_t Tab[(phi_t + j r_t + K_t j(j-1)/2) >> 48],
// each product and each partial sum rounded to FP32 in ascending tone order
// (no fused multiply-add: the DAC word below is decided by these roundings),
// then rounded to the nearest integer (ties to even) and saturated to int16,
// I and Q interleaved.  Tab is the DDC's FP32 cos/sin table; here it is read
// from a half-wave sine table in LDS, S[i] = sin(2 pi i / 2^16) for
// i < 2^15:  sin = +-S[i mod 2^15] (sign = bit 15 of i) and cos(i) =
// sin(i + 2^14), the same values and signs (zeros included) as the full table.
//
// Each thread produces kTxRun consecutive samples; the tone loop is uniform,
// so tone parameters come through the scalar cache.  The first work-group
// also writes the state after the buffer for the next call.
#include "rf_internal.hpp"

namespace rfk {

constexpr int kTxWG = 1024;
constexpr int kTxRun = 16;

__device__ __forceinline__ uint64_t tx_tri(uint64_t m)
{
    return (m & 1) ? m * ((m - 1) >> 1) : (m >> 1) * (m - 1);
}

__device__ __forceinline__ float tx_signed(uint32_t signsrc, float mag)
{
    return __uint_as_float((signsrc & 0x80000000u) | __float_as_uint(mag));
}

__device__ __forceinline__ uint32_t tx_dac(float v)
{
    float r = __builtin_rintf(v);
    r = fminf(fmaxf(r, -32768.0f), 32767.0f);
    return (uint32_t)(uint16_t)(int16_t)(int)r;
}

template <bool CHIRP>
__global__ void __launch_bounds__(kTxWG) tx_synth(TxLaunch a)
{
#pragma clang fp contract(off)
    __shared__ float stab[kSinTabLen];
    {
        const float4 *s4 = reinterpret_cast<const float4 *>(a.halftab);
        float4 *d4 = reinterpret_cast<float4 *>(stab);
        for (int i = threadIdx.x; i < kSinTabLen / 4; i += kTxWG) d4[i] = s4[i];
    }
    __syncthreads();
    const int64_t j0 = ((int64_t)blockIdx.x * kTxWG + threadIdx.x) * kTxRun;
    if (j0 < a.n) {
        const uint64_t uj = (uint64_t)j0;
        const uint64_t tj = CHIRP ? tx_tri(uj) : 0;
        float vr[kTxRun], vi[kTxRun];
#pragma unroll
        for (int b = 0; b < kTxRun; ++b) vr[b] = vi[b] = 0.0f;
        for (int t = 0; t < a.ntones; ++t) {
            const float amp = a.amp[t];
            uint64_t rate = a.rate[t];
            uint64_t ph = a.phase[t] + uj * rate;
            uint64_t K = 0;
            if constexpr (CHIRP) {
                K = a.chirp[t];
                ph += K * tj;
                rate += K * uj;
            }
#pragma unroll
            for (int b = 0; b < kTxRun; ++b) {
                const uint32_t hi = (uint32_t)(ph >> 32);
                const uint32_t hc = hi + 0x40000000u;   // a quarter turn on: cos = sin(. + pi/2)
                const float s = tx_signed(hi, stab[(hi >> 16) & 0x7fffu]);
                const float c = tx_signed(hc, stab[(hc >> 16) & 0x7fffu]);
                vr[b] = vr[b] + amp * c;
                vi[b] = vi[b] + amp * s;
                ph += rate;
                if constexpr (CHIRP) rate += K;
            }
        }
#pragma unroll
        for (int b = 0; b < kTxRun; ++b)
            if (j0 + b < a.n) a.out[j0 + b] = tx_dac(vr[b]) | (tx_dac(vi[b]) << 16);
    }
    if (blockIdx.x == 0) {
        const uint64_t n = (uint64_t)a.n;
        for (int t = threadIdx.x; t < a.ntones; t += kTxWG) {
            const uint64_t K = CHIRP ? a.chirp[t] : 0;
            a.phase_out[t] = a.phase[t] + n * a.rate[t] + K * tx_tri(n);
            a.rate_out[t] = a.rate[t] + n * K;
        }
    }
}

hipError_t launch_tx(const TxLaunch &a, hipStream_t s)
{
    if (a.n < 1 || a.ntones < 1) return hipErrorInvalidValue;
    const int64_t per = (int64_t)kTxWG * kTxRun;
    const int64_t grid = (a.n + per - 1) / per;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    if (a.chirp)
        hipLaunchKernelGGL(tx_synth<true>, dim3((unsigned)grid), dim3(kTxWG), 0, s, a);
    else
        hipLaunchKernelGGL(tx_synth<false>, dim3((unsigned)grid), dim3(kTxWG), 0, s, a);
    return hipGetLastError();
}

}  // namespace rfk
