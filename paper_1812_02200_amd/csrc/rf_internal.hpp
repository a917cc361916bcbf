// rf_internal.hpp -- launch interface between the C-ABI runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_device.hpp"

namespace rfk {

// Virtual stream seen by one process call: `hist` (H retained samples) followed
// by `in` (n new samples); sample v of the virtual stream is hist[v] for v < H,
// in[v - H] otherwise.  Samples are packed int16 I/Q words (I low, Q high).
struct VStream {
    const uint32_t *hist;
    const uint32_t *in;
    int64_t H;
    int64_t n;
};

struct PfbLaunch {
    VStream vs;
    uint32_t *hist_out;     // receives the new history (other ping-pong buffer)
    int64_t keep_from;      // virtual index of the first retained sample
    int64_t keep_len;       // number of retained samples
    float *out;             // [F x N] complex64
    const float *taps;      // [N*M]
    const float *tw;        // twiddle tables, float pairs, all passes
    int64_t F;              // frames to emit
    int32_t run_len;        // frames per lane-group run (multiple of 4)
    int32_t N, M;
    int32_t variant;        // kernel variant bits (0: default)
    const int32_t *sel;     // [nsel] chosen bins in output order, or null for all N bins
    int32_t nsel;           // output row length when sel is set
};

struct DdcLaunch {
    VStream vs;
    uint32_t *hist_out;
    int64_t keep_from;
    int64_t keep_len;
    float *out;             // tone-major, row stride ld complex values
    int64_t ld;
    const float *wrev;      // reversed taps: wrev[j] = h[T-1-j]
    const uint64_t *inc;    // [ntones]
    const uint64_t *phi0;   // [ntones]
    const uint64_t *chirp;  // [ntones] phase second differences (chirped tones), or null
    const float *sintab;    // quarter-wave (cos, sin) pair table, 2^14 pairs
    uint64_t base_abs;      // absolute sample index of virtual sample 0
    int64_t nout;           // outputs per tone this call
    uint64_t *phase_out;    // [ntones]: phi0 + phase_at * inc
    uint64_t phase_at;
    int32_t T, D, ntones;
    int32_t grid;           // work-groups to launch (persistent)
};

// Grouped launches: a device-side header and item table, rewritten between
// launches (the kernels read the count and the work-group total from memory,
// so a captured graph can be replayed for every batch).
struct GroupHeader {
    int32_t count;          // items
    int32_t pad;
    int64_t total;          // logical work-groups (PFB) or work units (DDC)
};

// A pointer loaded from device memory (an item table of a grouped launch)
// carries no address space, so accesses through it compile to flat
// instructions, which every LDS wait then also waits for.  Hot accesses go
// through a pointer typed in the global address space instead (a no-op
// where the compiler already knows it, as for kernel arguments).
#define RF_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ RF_GLOBAL T *gptr(T *p)
{
    return (RF_GLOBAL T *)p;
}

struct PfbItem {
    PfbLaunch a;
    int64_t wg_begin;       // first logical work-group of this item
    int32_t wgs;            // logical work-groups of this item
    int32_t pad;
};

// Logical work-groups a single-stream PFB launch of `a` uses.
int64_t pfb_launch_wgs(const PfbLaunch &a);
hipError_t launch_pfb_group(int N, int M, const GroupHeader *hdr, const PfbItem *items, int grid,
                            hipStream_t s);
int pfb_group_wg_size(int N);

// Fill n packed I/Q words with pseudo-random 14-bit values (tuning scratch).
hipError_t fill_iq(uint32_t *p, uint64_t n, hipStream_t s);

// Columns per thread in the fused PFB kernel, which is also the radix of the
// FFT pass done in the FIR's registers: 8 for N = 4096 (512-thread
// work-groups, so each thread keeps a 256-register budget), else 4.
__host__ __device__ constexpr int pfb_fir_radix(int N) { return N >= 4096 ? 8 : 4; }

// Twiddle table size (float pairs) for an N-point plan.
int pfb_twiddle_count(int N);
// Fill the twiddle table (host memory, float pairs) for an N-point plan.
void pfb_twiddle_fill(int N, float *tw);

hipError_t launch_pfb(const PfbLaunch &a, hipStream_t s);

// DFT on MFMA with hi/lo half-precision operands (N = 16 .. 256, powers of two).
// Variant bit 32 adds the lo*lo product term.
enum { RF_PREC_F16 = 1, RF_PREC_BF16 = 2 };
hipError_t launch_pfb_mfma(const PfbLaunch &a, int prec, hipStream_t s);
int pfb_mfma_table_floats();
// Exponent e of the exact tap scale 2^e that keeps every half-precision GEMM
// operand within 2^15 for any int16 input (false: no such e in [-100, 100]).
bool pfb_mfma_scale_exponent(const float *h, int N, int M, int *e);
void pfb_mfma_table_fill(int N, int scale_exp, float *t);
// Frames per run and launch geometry the PFB launcher will use.
int pfb_default_run_len(int N, int M, int64_t F);

hipError_t launch_ddc(const DdcLaunch &a, hipStream_t s);

struct DdcItem {
    DdcLaunch a;
    int64_t unit_begin;     // first work unit of this item in the table
    int64_t unit_off;       // its first unit within the call's units (a chunk of a long call)
    int64_t units;          // units of this item (the call's last unit is its tail)
};
// Threads (= tones per chunk) of the work-group that serves a bank of `ntones`
// (64 .. 1024, the same rule as the single-stream launch); a grouped launch
// holds items of one such size only.
int ddc_group_wg(int ntones);
// Work units of one item in a grouped launch: (tone chunk, output) pairs + 1 tail.
int64_t ddc_group_units(const DdcLaunch &a);
hipError_t launch_ddc_group(int wg, const GroupHeader *hdr, const DdcItem *items, int grid, hipStream_t s);
// The grouped kernels as function pointers (graph kernel nodes), or null.
const void *ddc_group_kernel(int wg);
const void *pfb_group_kernel(int N, int M);
int ddc_default_grid(int ntones, int64_t nout);

// Number of float entries of the half-wave sine table.
constexpr int kSinTabLen = 1 << 15;   // floats in the DDC oscillator table (2^14 cos/sin pairs)

// PFB for large or non-power-of-two N (pfb_large.hip).
struct LargePlan {
    int64_t N = 0;
    int N1 = 0, N2 = 1;      // N = N1 * N2, each <= 4096 (N2 = 1: one step)
    int nr1 = 0, nr2 = 0;    // radices of the two transform lengths
    int rad1[16] = {}, rad2[16] = {};
};
struct LargeBuffers {
    cf *v = nullptr;         // folded frames [frames x N]
    cf *y = nullptr;         // first-step output [frames x N]
    const float *tables = nullptr;   // W_N1^j, W_N2^j, then the three W_N tables
};
struct StepDesc {
    int L, nr, TB;
    int rad[16];
    const cf *tw;            // W_L^j
    int64_t C;               // transforms per frame
    int64_t in_cs, in_es, out_cs, out_es;
    const cf *t3;            // four-step twiddle tables (3 x 256, staged in LDS), or null:
                             // W_N^e = t3[512 + (e >> 16)] * t3[256 + ((e >> 8) & 255)] * t3[e & 255]
    const cf *src;
    cf *dst;
};
bool large_plan(int64_t N, LargePlan *pl);
bool large_supported(int64_t N);
size_t large_table_floats(const LargePlan &pl);
void large_table_fill(const LargePlan &pl, float *t);
hipError_t launch_pfb_large(const PfbLaunch &a, const LargePlan &pl, const LargeBuffers &b, hipStream_t s);

// Transmit synthesis (tx_kernels.hip).
struct TxLaunch {
    uint32_t *out;          // [n] int16 I/Q pairs (I low half)
    int64_t n;
    const uint64_t *phase;  // [ntones] oscillator state at the first sample
    const uint64_t *rate;
    const uint64_t *chirp;  // [ntones] second differences, or null
    const float *amp;       // [ntones] DAC counts
    const float *halftab;   // 2^15 floats: sin(2 pi i / 2^16), i < 2^15
    uint64_t *phase_out;    // [ntones] state after the buffer
    uint64_t *rate_out;
    int32_t ntones;
};
hipError_t launch_tx(const TxLaunch &a, hipStream_t s);

}  // namespace rfk
