// pfb_kernels.hpp -- fused int16 unpack + polyphase FIR + FFT for gfx950.
//
// Critically sampled polyphase filter bank (paper Sec. III.A): frame p of an
// N-channel bank with M taps per channel is
//     v_p[n] = sum_m h[mN+n] x[pN+mN+n],   X_p[k] = sum_n v_p[n] exp(-2 pi i kn/N).
// The paper folds with a cuBLAS product and transforms with batched cuFFT; here
// one kernel reads every input sample once from HBM, keeps the FIR's sliding
// window in registers and runs the FFT through LDS, writing only the spectra.
//
// Work decomposition (all compile-time in N):
//  * A lane group (LG) of L = N/C threads walks a contiguous run of frames
//    (C = 4 columns per thread; 8 for N = 4096, whose lane group is then a
//    512-thread work-group with 256 registers per thread instead of a
//    1024-thread one with 128).  Thread c of an LG owns the C columns
//    n = c + k*L (k < C), holds their M taps (for C = 8: in LDS or read
//    through the caches) and a window of M+FP-1 blocks of input in
//    registers, and produces FP frames per phase (4; 2 for C = 8).  Its C
//    FIR outputs are exactly the inputs of one radix-C butterfly of the
//    first Stockham pass (stride N/C, no twiddles), which it computes before
//    writing to LDS.
//  * The remaining passes are radix-16 (radix 8/4/2 for the last one) Stockham
//    passes: a team of N/16 threads owns one frame, every thread holds 16
//    points (or more, in several butterflies) per pass; the FP frames of a
//    phase buffer take the whole work-group.  The last pass writes the
//    natural-order spectrum straight to HBM
//    -- or, when the caller chose a set of channels, back to LDS, from where
//    the frame's team gathers the chosen bins into consecutive columns (same
//    arithmetic, fewer bytes written).
//  * LDS holds the frames of one phase, indexed with one float2 of padding per
//    32 entries (i + (i>>5)): the FIR's radix-C outputs, C consecutive
//    entries per lane (lanes 8C bytes apart), and the strided stores of the
//    Stockham passes then hit distinct banks.  Pass twiddles are staged in LDS
//    as [r][k] tables so that lanes with consecutive k read consecutive entries.
//  * Work-groups whose every input block lies inside the new buffer (all but
//    the first and last few) take a branch-free path with a per-run base
//    pointer; the others resolve each block against the retained history.
//  * Work-groups are remapped so that each of the 8 XCDs walks one contiguous
//    part of the stream; neighbouring runs, which share M-1 blocks of input,
//    then meet in the same L2.
//
// Variant bits (kernel template parameter V, chosen at launch):
//   1: two LDS phase buffers, one work-group barrier per phase (N <= 1024);
//   2: ordinary (write-back) stores instead of non-temporal stores;
//   8: only chosen channels are stored (bin list in PfbLaunch::sel);
//  16: even work-groups walk their run backwards, so that neighbouring runs
//      read their shared blocks together (fast path; same results).
#pragma once
#include "fft_device.hpp"
#include "rf_internal.hpp"

namespace rfk {

typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Threads that transform one frame in the LDS passes.
__host__ __device__ constexpr int pfb_fft_team(int N) { return N / 16; }

// Frames a lane group produces per phase: 4, or 2 with eight columns per
// thread (the window of M+FP-1 blocks and the FIR's sums then fit in the
// register budget at M = 8).
__host__ __device__ constexpr int pfb_frames_per_phase(int N) { return pfb_fir_radix(N) == 8 ? 2 : 4; }

template <int N>
struct PfbPlan {
    static constexpr int C = pfb_fir_radix(N);      // columns per thread
    static constexpr int L = N / C;                  // threads per lane group
    static constexpr int WG = L > 256 ? L : 256;     // threads per work-group
    static constexpr int NLG = WG / L;               // lane groups per work-group
    static constexpr int FP = pfb_frames_per_phase(N);   // frames per lane group and phase
    static constexpr int FB = NLG * FP;              // frames per phase buffer
    static constexpr int NT = pfb_fft_team(N);       // FFT team size (threads)
    static_assert(NT * FB == WG, "one team per frame of the phase buffer");
    static constexpr int LDS = FB * N + ((FB * N) >> 5);
    static constexpr bool LG_IN_WAVE = L <= 64;      // FIR and FFT of an LG stay in one wave
    static constexpr bool TEAM_IN_WAVE = NT <= 64;
};

__host__ __device__ constexpr int pass_radix(int N, int NS) { return (N / NS) >= 16 ? 16 : (N / NS); }

// Pass twiddles, all staged in LDS.  Every pass but one has its full [r][k]
// table, W_{NS R}^{k r}.  The radix-2 last pass of N = 4096 would need 2048
// entries more than LDS holds; its butterfly j = tl + b*NT (k = j) takes
// W_N^j = W_N^tl * W_N^(b NT), from two factor tables of NT and N/(2 NT)
// entries.
template <int N, int NS>
struct TwPlace {
    static constexpr int R = pass_radix(N, NS);
    static constexpr bool FULL = (R == 16) || (N <= 2048);
};

// Table entries (float pairs) of the pass with stride ns.
__host__ __device__ constexpr int pass_tw_count(int N, int ns)
{
    const int R = pass_radix(N, ns);
    if (R == 16 || N <= 2048) return ns * R;
    const int nt = pfb_fft_team(N);
    return nt + (N / R) / nt;
}

// Offset (in float pairs) of the twiddle table of the pass with stride NS.
__host__ __device__ constexpr int tw_offset(int N, int NS)
{
    int off = 0;
    for (int ns = pfb_fir_radix(N); ns < NS; ns *= pass_radix(N, ns)) off += pass_tw_count(N, ns);
    return off;
}

template <int N>
__host__ __device__ constexpr int lds_tw_count()
{
    const int n = tw_offset(N, N);
    return n > 0 ? n : 1;
}

__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

// The value, hidden from the optimiser when ON: addresses derived from it
// inside a loop are then formed where they are used instead of being hoisted
// out of the loop and held (or spilled) across it.  (An index, not a
// pointer: a laundered pointer loses its address space and its loads become
// flat loads, which LDS waits then also wait for.)
template <bool ON, typename T>
__device__ __forceinline__ T phase_local(T x)
{
    if constexpr (ON) asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ void wave_fence()
{
    // LDS accesses of one wave complete in issue order; keep the compiler from
    // moving them across this point.
    __asm__ __volatile__("" ::: "memory");
}

template <bool CROSS_WAVE>
__device__ __forceinline__ void group_sync()
{
    if constexpr (CROSS_WAVE)
        __syncthreads();
    else
        wave_fence();
}

__device__ __forceinline__ uint32_t vload(const VStream &vs, int64_t v)
{
    return v < vs.H ? gptr(vs.hist)[v] : gptr(vs.in)[v - vs.H];
}

__device__ __forceinline__ cf unpack(uint32_t w)
{
    return {(float)(int16_t)(w & 0xffffu), (float)(int16_t)(w >> 16)};
}

// Load the C columns c + k*L of virtual block b (samples [bN, bN+N)),
// resolving each against history, new input and end of data.
template <int N>
__device__ __forceinline__ void load_block(const VStream &vs, int64_t vlen, int64_t b, int c,
                                           uint32_t (&w)[pfb_fir_radix(N)])
{
    constexpr int C = pfb_fir_radix(N);
    constexpr int L = N / C;
    const int64_t base = b * N;
    if (base + N <= vlen) {
        if (base >= vs.H) {
            const RF_GLOBAL uint32_t *p = gptr(vs.in) + (base - vs.H) + c;
#pragma unroll
            for (int k = 0; k < C; ++k) w[k] = p[k * L];
        } else if (base + N <= vs.H) {
            const RF_GLOBAL uint32_t *p = gptr(vs.hist) + base + c;
#pragma unroll
            for (int k = 0; k < C; ++k) w[k] = p[k * L];
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) w[k] = vload(vs, base + c + k * L);
        }
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            int64_t v = base + c + k * L;
            w[k] = v < vlen ? vload(vs, v) : 0u;
        }
    }
}

// One Stockham pass of radix R and stride NS over the frame at `fb` (LDS,
// unpadded frame base).  Thread `tl` of the frame's team handles butterflies
// j = tl + b*NT.  The last pass stores to `outf` (global, frame base), or,
// with SEL (chosen channels), back to LDS in natural bin order.
template <int N, int R, int NS, bool LAST, bool NT_STORE, bool SEL>
__device__ __forceinline__ void fft_pass(cf *lds, int fb, int tl, const cf *twl, RF_GLOBAL float *__restrict__ outf,
                                         bool valid, const RF_GLOBAL int32_t *__restrict__ sel)
{
    constexpr int NT = PfbPlan<N>::NT;
    constexpr int NB = N / R;
    constexpr int BPT = NB / NT;
    constexpr bool XW = !PfbPlan<N>::TEAM_IN_WAVE;
    constexpr int TOFF = tw_offset(N, NS);
    static_assert(BPT * NT == NB, "team does not tile the pass");
    cf v[BPT][R];
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int j = tl + b * NT;
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = lds[lpad(fb + j + r * NB)];
    }
    group_sync<XW>();
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
        const int j = tl + b * NT;
        const int k = j % NS;
        if constexpr (NS > 1) {
            if constexpr (TwPlace<N, NS>::FULL) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], twl[TOFF + r * NS + k]);
            } else {
                static_assert(R == 2 && NS * R == N, "factor tables serve the radix-2 last pass");
                v[b][1] = cmul(v[b][1], cmul(twl[TOFF + tl], twl[TOFF + NT + b]));
            }
        }
        dft<R>(v[b]);
        const int idxD = (j / NS) * NS * R + k;
        if constexpr (LAST && !SEL) {
            if (valid) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    f2v o = {v[b][r].x, v[b][r].y};
                    RF_GLOBAL f2v *dst = (RF_GLOBAL f2v *)(outf + 2 * (idxD + r * NS));
                    if constexpr (NT_STORE)
                        __builtin_nontemporal_store(o, dst);
                    else
                        *dst = o;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < R; ++r) lds[lpad(fb + idxD + r * NS)] = v[b][r];
        }
    }
    if constexpr (!LAST) group_sync<XW>();
}

// STAGED: the last pass leaves the spectrum in LDS (natural bin order) for
// the caller to copy out.
template <int N, int NS, bool NT_STORE, bool SEL, bool STAGED = false>
__device__ __forceinline__ void fft_passes(cf *lds, int fb, int tl, const cf *twl, RF_GLOBAL float *__restrict__ outf,
                                           bool valid, const RF_GLOBAL int32_t *__restrict__ sel, int nsel)
{
    if constexpr (NS < N) {
        constexpr int R = pass_radix(N, NS);
        fft_pass<N, R, NS, NS * R == N, NT_STORE, SEL || STAGED>(lds, fb, tl, twl, outf, valid, sel);
        fft_passes<N, NS * R, NT_STORE, SEL, STAGED>(lds, fb, tl, twl, outf, valid, sel, nsel);
    } else if constexpr (SEL) {
        // the spectrum is in LDS: the team gathers the chosen bins into
        // consecutive columns (sel = the bins, in output order)
        group_sync<!PfbPlan<N>::TEAM_IN_WAVE>();
        if (valid) {
            for (int c = tl; c < nsel; c += PfbPlan<N>::NT) {
                const cf x = lds[lpad(fb + sel[c])];
                f2v o = {x.x, x.y};
                RF_GLOBAL f2v *dst = (RF_GLOBAL f2v *)(outf + 2 * c);
                if constexpr (NT_STORE)
                    __builtin_nontemporal_store(o, dst);
                else
                    *dst = o;
            }
        }
    }
}

// Window element: unpacked FP32 pair, or the raw packed word for large M
// (fewer registers, one conversion per use).
template <bool PACKED>
struct WinT;
template <>
struct WinT<false> {
    cf v;
    __device__ __forceinline__ void set(uint32_t w) { v = unpack(w); }
    __device__ __forceinline__ cf get() const { return v; }
};
template <>
struct WinT<true> {
    uint32_t w;
    __device__ __forceinline__ void set(uint32_t x) { w = x; }
    __device__ __forceinline__ cf get() const { return unpack(w); }
};

// Eight columns per thread (N = 4096): M x 8 taps would not fit beside the
// window.  The handle stores a copy [m][q][c][4] (tap m of thread c's
// columns 4q .. 4q+3, 16 bytes; consecutive threads at consecutive 16-byte
// slots, so one wave's row read is 1 KiB contiguous) after the natural
// [m N + n] layout.  For M <= 4 each
// thread copies its rows into LDS (64 KiB at most, read only by that thread);
// otherwise every phase reads them from that copy, through the caches (all
// work-groups of an XCD read the same taps).  (Measured: splitting larger M
// between LDS and memory, or keeping some rows in registers, made the
// compiler hoist more and ran slower.)  Every sum adds its M terms in tap
// order either way.
template <int N>
struct TapsInMemory {
    static constexpr bool ON = pfb_fir_radix(N) == 8;
};

template <int N, int M>
struct TapTiers {
    static constexpr int LR = TapsInMemory<N>::ON && M <= 4 ? M : 0;   // rows in LDS
    static constexpr int LDS_F4 = LR * 2 * (N / 8);                  // LDS float4 entries
};

template <int N, int M>
struct FirState {
    static constexpr int C = pfb_fir_radix(N);
    static constexpr bool PACKED = (M > 8) || (C == 8);
    static constexpr int FP = pfb_frames_per_phase(N);
    static constexpr int W = M + FP - 1;   // window blocks fp .. fp+M+FP-2
    float hr[TapsInMemory<N>::ON ? 1 : M][C];
    const RF_GLOBAL f4v *tp;          // TapsInMemory: row m, part q of this thread's taps at tp[(2 m + q) L]
    const f4v *tl;                    // TapsInMemory: the same in LDS
    WinT<PACKED> xw[W][C];
};

// FIR of the phase's FP frames, first radix-C pass, store to LDS.
template <int N, int M>
__device__ __forceinline__ void fir_phase(const FirState<N, M> &st, cf *lds, int g, int c)
{
    constexpr int C = FirState<N, M>::C;
    constexpr int FP = FirState<N, M>::FP;
    if constexpr (TapsInMemory<N>::ON) {
        // taps outer: each row of C taps is read once and applied to the FP
        // frames; every sum still adds its M terms in tap order
        cf s[FP][C];
#pragma unroll
        for (int qf = 0; qf < FP; ++qf)
#pragma unroll
            for (int k = 0; k < C; ++k) s[qf][k] = cf{0.f, 0.f};
        using TT = TapTiers<N, M>;
        constexpr int L = N / C;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            float t[C];
#pragma unroll
            for (int q = 0; q < C / 4; ++q) {
                const f4v t4 = m < TT::LR ? st.tl[(m * (C / 4) + q) * L] : st.tp[(m * (C / 4) + q) * L];
                t[4 * q] = t4.x;
                t[4 * q + 1] = t4.y;
                t[4 * q + 2] = t4.z;
                t[4 * q + 3] = t4.w;
            }
#pragma unroll
            for (int qf = 0; qf < FP; ++qf)
#pragma unroll
                for (int k = 0; k < C; ++k) {
                    // each use converts afresh: converted copies kept for
                    // the block's second use would cost two registers per word
                    uint32_t w = st.xw[qf + m][k].w;
                    asm volatile("" : "+v"(w));
                    const cf x = unpack(w);
                    s[qf][k].x = __builtin_fmaf(t[k], x.x, s[qf][k].x);
                    s[qf][k].y = __builtin_fmaf(t[k], x.y, s[qf][k].y);
                }
        }
#pragma unroll
        for (int qf = 0; qf < FP; ++qf) {
            dft<C>(s[qf]);
            cf *dst = lds + lpad((g * FP + qf) * N + C * c);
#pragma unroll
            for (int r = 0; r < C; ++r) dst[r] = s[qf][r];
        }
        return;
    }
#pragma unroll
    for (int qf = 0; qf < FP; ++qf) {
        cf v[C];
#pragma unroll
        for (int k = 0; k < C; ++k) {
            cf s = {0.f, 0.f};
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const cf x = st.xw[qf + m][k].get();
                s.x = __builtin_fmaf(st.hr[m][k], x.x, s.x);
                s.y = __builtin_fmaf(st.hr[m][k], x.y, s.y);
            }
            v[k] = s;
        }
        dft<C>(v);
        // entries Cc .. Cc+C-1 never straddle a padding point (every 32)
        cf *dst = lds + lpad((g * FP + qf) * N + C * c);
#pragma unroll
        for (int r = 0; r < C; ++r) dst[r] = v[r];
    }
}

template <int N, int M>
__device__ __forceinline__ void shift_window(FirState<N, M> &st,
                                             const uint32_t (&pre)[pfb_frames_per_phase(N)][pfb_fir_radix(N)])
{
    constexpr int W = FirState<N, M>::W;
    constexpr int C = FirState<N, M>::C;
    constexpr int FP = FirState<N, M>::FP;
#pragma unroll
    for (int i = 0; i + FP < W; ++i)
#pragma unroll
        for (int k = 0; k < C; ++k) st.xw[i][k] = st.xw[i + FP][k];
#pragma unroll
    for (int i = 0; i < FP; ++i)
#pragma unroll
        for (int k = 0; k < C; ++k) st.xw[W - FP + i][k].set(pre[i][k]);
}

// Small N: a frame's team is a few threads (one for N = 16), so stores
// straight from the last pass would put 8-byte pieces of many frames into each
// wave store.  The spectra stay in LDS instead and each wave writes out its
// own lane groups' four frames (4N consecutive values in the output) with
// consecutive lanes on consecutive values.  Frames at or past the end of a
// lane group's run are not written.  (Measured: 6x faster at N = 16, 5% at
// N = 128, slower from N = 256 on, where a team's stores already cover whole
// 512-byte runs.)
template <int N>
struct PfbStage {
    static constexpr bool ON = N <= 128;
};

template <int N, bool NT_STORE>
__device__ __forceinline__ void staged_copy(const cf *lds, float *__restrict__ out, int64_t lg_base, int RL,
                                            int ph, int64_t F)
{
    constexpr int L = PfbPlan<N>::L;
    static_assert(L <= 64 && 64 % L == 0, "lane groups inside one wave");
    static_assert(PfbPlan<N>::FP == 4, "four frames per phase");
    constexpr int LGW = 64 / L;   // lane groups per wave
    constexpr int CH = 4 * N;     // values of a lane group's four frames
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll 1
    for (int i = 0; i < LGW; ++i) {
        const int g = wv * LGW + i;
        const int64_t run0 = (lg_base + g) * RL;
        const int64_t f1 = run0 + RL < F ? run0 + RL : F;
        const int64_t fg = run0 + 4 * ph;
#pragma unroll
        for (int e = lane; e < CH; e += 64) {
            if (fg + e / N < f1) {
                const cf x = lds[lpad(4 * g * N + e)];
                f2v o = {x.x, x.y};
                RF_GLOBAL f2v *dst = (RF_GLOBAL f2v *)(gptr(out) + 2 * (fg * N + e));
                if constexpr (NT_STORE)
                    __builtin_nontemporal_store(o, dst);
                else
                    *dst = o;
            }
        }
    }
}

template <int N, int V>
struct PfbVariant {
    static constexpr bool DBUF = (V & 1) && N <= 1024 && !PfbPlan<N>::LG_IN_WAVE;
    static constexpr bool NT_STORE = !(V & 2);
    static constexpr int NBUF = DBUF ? 2 : 1;
};

// LDS of the PFB body, sized for its plan, variant and tap count.
template <int N, int V, int M>
struct PfbShared {
    cf frames[PfbVariant<N, V>::NBUF * PfbPlan<N>::LDS];
    cf tw[lds_tw_count<N>()];
    f4v taps[TapTiers<N, M>::LDS_F4 > 0 ? TapTiers<N, M>::LDS_F4 : 1];   // [m][q][c]
};

// The whole PFB computation of one logical work-group `lwg` of `G` for the
// call described by `a`.  Shared by the single-stream kernel and the grouped
// multi-stream kernel, so a stream's frames are computed by the same
// instructions either way.  OPAQUE (callers that run the body in a loop):
// the thread index is hidden from the optimiser, so each run's per-thread
// addresses are computed in it instead of being kept live across runs.
template <int N, int M, int V, bool OPAQUE = false>
__device__ __forceinline__ void pfb_body(const PfbLaunch &a, int lwg, int G, PfbShared<N, V, M> &sh)
{
    using P = PfbPlan<N>;
    using VV = PfbVariant<N, V>;
    constexpr int L = P::L;
    constexpr int C = P::C;
    constexpr int FP = P::FP;
    constexpr int W = FirState<N, M>::W;
    constexpr int TWL = lds_tw_count<N>();
    // one barrier per phase when double buffered, else two
    constexpr bool SYNC2 = !P::LG_IN_WAVE && !VV::DBUF;
    // eight columns per thread: the FFT's per-thread addresses (16 stores and
    // twiddles per pass) are recomputed in each phase rather than kept live
    constexpr bool RELOAD = C == 8;
    // The next phase's input is requested before the FIR, except where the
    // FIR reads its taps from memory: loads complete in order, so the tap
    // loads would wait for the prefetch; it follows the FIR instead.  These
    // blocks are read by this run only (a run shares only its first and last
    // M-1 blocks with its neighbours, which its window loads read): they are
    // loaded non-temporally, so they do not displace shared blocks in the L2
    // (measured 2-3 us faster per 2^24-sample launch at N = 1024, M = 8).
    constexpr bool PRE_AFTER = TapsInMemory<N>::ON;
    // Short runs of small frames (N <= 64: tuned runs of 8 to 16 frames
    // against M-1 shared blocks at each edge) keep the shared edge blocks in
    // ordinary loads (N = 16, M = 8: 57 -> 51 us per 2^24 samples); from
    // N = 128 on, streaming every prefetched block measured as fast or faster
    // (N = 1024: 45 against 48 us).
    constexpr bool EDGE_CACHED = N <= 64;
    cf *lds_all = sh.frames;
    cf *twl = sh.tw;

    int tid = threadIdx.x;
    if constexpr (OPAQUE) {
        asm volatile("" : "+v"(tid));
        __builtin_assume(tid >= 0 && tid < P::WG);
    }
    const RF_GLOBAL f2v *twg = reinterpret_cast<const RF_GLOBAL f2v *>(gptr(a.tw));
    for (int i = tid; i < TWL; i += P::WG) {
        const f2v t = twg[i];
        twl[i] = cf{t.x, t.y};
    }

    const VStream vs = a.vs;
    const int64_t vlen = vs.H + vs.n;
    const int64_t F = a.F;
    const int RL = a.run_len;
    const int nph = RL / FP;
    // output row length: all N bins, or the chosen channels (variant bit 8:
    // a.sel lists the bins in output order; compiled only into that variant)
    constexpr bool SEL = (V & 8) != 0;
    constexpr bool STAGE = PfbStage<N>::ON && !SEL;
    const RF_GLOBAL int32_t *sel = SEL ? gptr(a.sel) : nullptr;
    const int64_t ldo = SEL ? (int64_t)a.nsel : (int64_t)N;

    const int g = tid / L;
    const int c = tid - g * L;
    const int64_t f0 = ((int64_t)lwg * P::NLG + g) * RL;

    // Every block this work-group touches lies inside the new input: no
    // history, no tail, every frame valid.  Uniform per work-group.
    const int64_t wg_first = (int64_t)lwg * P::NLG * RL;
    const int64_t wg_last = wg_first + (int64_t)P::NLG * RL + M - 2;
    const bool fast = wg_first * N >= vs.H && (wg_last + 1) * N <= vlen;

    FirState<N, M> st;
    if constexpr (TapsInMemory<N>::ON) {
        using TT = TapTiers<N, M>;
        st.tp = reinterpret_cast<const RF_GLOBAL f4v *>(gptr(a.taps) + (size_t)N * M) + c;
        st.tl = sh.taps + c;
#pragma unroll
        for (int m = 0; m < TT::LR; ++m)
#pragma unroll
            for (int q = 0; q < C / 4; ++q) sh.taps[(m * (C / 4) + q) * L + c] = st.tp[(m * (C / 4) + q) * L];
    } else {
#pragma unroll
        for (int m = 0; m < M; ++m)
#pragma unroll
            for (int k = 0; k < C; ++k) st.hr[m][k] = gptr(a.taps)[m * N + c + k * L];
    }

    // FFT team of this thread (may belong to another lane group for N >= 512)
    const int slot = tid / P::NT;
    const int tl = tid - slot * P::NT;
    const int lg2 = slot / FP, q2 = slot - lg2 * FP;
    const int64_t f0t = ((int64_t)lwg * P::NLG + lg2) * RL;
    const int64_t f1t = (f0t + RL < F) ? f0t + RL : F;
    __syncthreads();   // twiddle tables staged

    if constexpr ((V & 16) != 0) {
        if (fast) {
            // Variant bit 16: even runs are walked backwards (last phase
            // first), so two neighbouring runs read the M-1 blocks they share
            // at about the same time and the second read hits the cache.  Each
            // frame's sum is formed exactly as in the forward walk.  (A lane
            // group is at least one whole wave here, N >= 256, so the choice
            // is uniform per wave.)
            static_assert(P::L >= 64, "lane groups of whole waves");
            const bool back = (((int64_t)lwg * P::NLG + g) & 1) == 0;
            const RF_GLOBAL uint32_t *base = gptr(vs.in) + (f0 * N - vs.H) + c;
            const int64_t b0 = back ? FP * (int64_t)(nph - 1) : 0;   // first window block
#pragma unroll
            for (int i = 0; i < W; ++i)
#pragma unroll
                for (int k = 0; k < C; ++k) st.xw[i][k].set(base[(b0 + i) * N + k * L]);
#pragma unroll 1
            for (int it = 0; it < nph; ++it) {
                const int ph = back ? nph - 1 - it : it;
                cf *lds = lds_all + (VV::DBUF ? (it & 1) * P::LDS : 0);
                uint32_t pre[FP][C];
                const bool more = it + 1 < nph;
                auto prefetch = [&]() __attribute__((always_inline)) {
                    if (more) {
                        const RF_GLOBAL uint32_t *p = (base - c) + phase_local<RELOAD>(c) + (int64_t)(back ? FP * ph - FP : FP * ph + W) * N;
                        // blocks read by this run only stream; with EDGE_CACHED the
                        // blocks it shares with the neighbouring run (within M-1
                        // of the run's edge) stay cached
                        auto stream = [&]() __attribute__((always_inline)) {
#pragma unroll
                            for (int i = 0; i < FP; ++i)
#pragma unroll
                                for (int k = 0; k < C; ++k) pre[i][k] = __builtin_nontemporal_load(&p[i * N + k * L]);
                        };
                        if constexpr (!EDGE_CACHED) {
                            stream();
                        } else if (back ? FP * ph - FP >= M - 1 : FP * ph + W + FP <= RL) {
                            stream();
                        } else {
#pragma unroll
                            for (int i = 0; i < FP; ++i)
#pragma unroll
                                for (int k = 0; k < C; ++k) pre[i][k] = p[i * N + k * L];
                        }
                    }
                };
                if constexpr (!PRE_AFTER) prefetch();
                fir_phase<N, M>(st, lds, g, c);
                if constexpr (PRE_AFTER) prefetch();
                group_sync<!P::LG_IN_WAVE>();
                fft_passes<N, C, VV::NT_STORE, SEL, STAGE>(lds, slot * N, phase_local<RELOAD>(tl), twl,
                                                      gptr(a.out) + 2 * (f0t + FP * ph + q2) * ldo, true, sel,
                                                      a.nsel);
                if constexpr (STAGE) {
                    wave_fence();
                    staged_copy<N, VV::NT_STORE>(lds, a.out, (int64_t)lwg * P::NLG, RL, ph, F);
                }
                if constexpr (SYNC2) group_sync<true>();
                else wave_fence();
                if (more) {
                    if (back) {
#pragma unroll
                        for (int i = W - 1; i >= FP; --i)
#pragma unroll
                            for (int k = 0; k < C; ++k) st.xw[i][k] = st.xw[i - FP][k];
#pragma unroll
                        for (int i = 0; i < FP; ++i)
#pragma unroll
                            for (int k = 0; k < C; ++k) st.xw[i][k].set(pre[i][k]);
                    } else {
                        shift_window<N, M>(st, pre);
                    }
                }
            }
        }
    }
    if (fast && (V & 16) == 0) {
        // block b of this lane group starts at in + (f0 + b)*N - H
        const RF_GLOBAL uint32_t *base = gptr(vs.in) + (f0 * N - vs.H) + c;
#pragma unroll
        for (int i = 0; i < W; ++i)
#pragma unroll
            for (int k = 0; k < C; ++k) st.xw[i][k].set(base[i * N + k * L]);
        auto phase = [&](int ph) __attribute__((always_inline)) {
            cf *lds = lds_all + (VV::DBUF ? (ph & 1) * P::LDS : 0);
            uint32_t pre[FP][C];
            const bool more = ph + 1 < nph;
            auto prefetch = [&]() __attribute__((always_inline)) {
                if (more) {
                    const RF_GLOBAL uint32_t *p = (base - c) + phase_local<RELOAD>(c) + (int64_t)(FP * ph + W) * N;
                    auto stream = [&]() __attribute__((always_inline)) {   // blocks read by this run only
#pragma unroll
                        for (int i = 0; i < FP; ++i)
#pragma unroll
                            for (int k = 0; k < C; ++k) pre[i][k] = __builtin_nontemporal_load(&p[i * N + k * L]);
                    };
                    if constexpr (!EDGE_CACHED) {
                        stream();
                    } else if (FP * ph + W + FP <= RL) {
                        stream();
                    } else {                        // shared with the next run: keep them cached
#pragma unroll
                        for (int i = 0; i < FP; ++i)
#pragma unroll
                            for (int k = 0; k < C; ++k) pre[i][k] = p[i * N + k * L];
                    }
                }
            };
            if constexpr (!PRE_AFTER) prefetch();
            fir_phase<N, M>(st, lds, g, c);
            if constexpr (PRE_AFTER) prefetch();
            group_sync<!P::LG_IN_WAVE>();
            fft_passes<N, C, VV::NT_STORE, SEL, STAGE>(lds, slot * N, phase_local<RELOAD>(tl), twl,
                                                  gptr(a.out) + 2 * (f0t + FP * ph + q2) * ldo, true, sel, a.nsel);
            if constexpr (STAGE) {
                wave_fence();
                staged_copy<N, VV::NT_STORE>(lds, a.out, (int64_t)lwg * P::NLG, RL, ph, F);
            }
            if constexpr (SYNC2) group_sync<true>();
            else wave_fence();
            if (more) shift_window<N, M>(st, pre);
        };
        // Three phases bring in 3 FP blocks; when that is at least the window
        // (M <= 2 FP + 1), no window value survives to the loop edge of a
        // group of three and the window needs no register rotation there (a
        // move per value).
        int ph = 0;
        for (; ph + 3 <= nph; ph += 3) {
            phase(ph);
            phase(ph + 1);
            phase(ph + 2);
        }
        for (; ph < nph; ++ph) phase(ph);
    } else if (!fast) {
#pragma unroll
        for (int i = 0; i < W; ++i) {
            uint32_t w[C];
            load_block<N>(vs, vlen, f0 + i, c, w);
#pragma unroll
            for (int k = 0; k < C; ++k) st.xw[i][k].set(w[k]);
        }
        for (int ph = 0; ph < nph; ++ph) {
            cf *lds = lds_all + (VV::DBUF ? (ph & 1) * P::LDS : 0);
            const int64_t fp = f0 + FP * ph;
            uint32_t pre[FP][C];
            const bool more = (ph + 1 < nph) && (fp + FP < F);
            auto prefetch = [&]() __attribute__((always_inline)) {
                if (more) {
#pragma unroll
                    for (int i = 0; i < FP; ++i) load_block<N>(vs, vlen, fp + W + i, c, pre[i]);
                }
            };
            if constexpr (!PRE_AFTER) prefetch();
            if (fp < F) fir_phase<N, M>(st, lds, g, c);
            if constexpr (PRE_AFTER) prefetch();
            group_sync<!P::LG_IN_WAVE>();
            {
                const int64_t f = f0t + FP * ph + q2;
                const bool valid = f < f1t;
                fft_passes<N, C, VV::NT_STORE, SEL, STAGE>(lds, slot * N, phase_local<RELOAD>(tl), twl,
                                                      gptr(a.out) + 2 * (valid ? f : 0) * ldo, valid, sel, a.nsel);
            }
            if constexpr (STAGE) {
                wave_fence();
                staged_copy<N, VV::NT_STORE>(lds, a.out, (int64_t)lwg * P::NLG, RL, ph, F);
            }
            if constexpr (SYNC2) group_sync<true>();
            else wave_fence();
            if (more) shift_window<N, M>(st, pre);
        }
    }

    // retained history for the next call (sources are read-only this call)
    for (int64_t i = (int64_t)lwg * P::WG + tid; i < a.keep_len; i += (int64_t)G * P::WG)
        gptr(a.hist_out)[i] = vload(vs, a.keep_from + i);
}

template <int N, int M, int V>
__global__ void __launch_bounds__(PfbPlan<N>::WG) __attribute__((amdgpu_waves_per_eu(M <= 8 ? 2 : 1))) pfb_fir_fft(PfbLaunch a)
{
    __shared__ PfbShared<N, V, M> sh;
    // XCD-aware work-group order: blocks are dealt round-robin to the 8 XCDs,
    // so give XCD x the contiguous logical range [x*q + min(x,r), ...).
    const int G = gridDim.x, bid = blockIdx.x;
    const int xq = G >> 3, xr = G & 7, xcd = bid & 7;
    const int lwg = xcd * xq + (xcd < xr ? xcd : xr) + (bid >> 3);
    pfb_body<N, M, V>(a, lwg, G, sh);
}

// Grouped launch: the buffers of many streams with the same (N, M) in one
// grid.  Work-groups stride over the concatenated logical work-groups of all
// items (a persistent grid), each item keeping its own history, taps and
// output.  The item table lives in device memory and is rewritten between
// launches, so one captured graph serves every batch.
template <int N, int M>
__global__ void __launch_bounds__(PfbPlan<N>::WG) __attribute__((amdgpu_waves_per_eu(M <= 8 ? 2 : 1)))
pfb_group(const GroupHeader *hdr, const PfbItem *items)
{
    __shared__ PfbShared<N, 0, M> sh;
    const int nitems = hdr->count;
    const int64_t total = hdr->total;
    for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
        int lo = 0, hi = nitems - 1;       // last item with wg_begin <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].wg_begin <= w) lo = mid;
            else hi = mid - 1;
        }
        const PfbItem &it = items[lo];
        pfb_body<N, M, 0, true>(it.a, (int)(w - it.wg_begin), it.wgs, sh);
        __syncthreads();   // LDS is reused by the next item
    }
}

// Logical work-groups of one call (at least one, for the history copy).
template <int N>
inline int64_t pfb_wgs(const PfbLaunch &a)
{
    const int64_t runs = (a.F + a.run_len - 1) / a.run_len;
    int64_t wgs = (runs + PfbPlan<N>::NLG - 1) / PfbPlan<N>::NLG;
    return wgs < 1 ? 1 : wgs;
}

template <int N, int M, int V>
hipError_t launch_pfb_nmv(const PfbLaunch &a, hipStream_t s)
{
    using P = PfbPlan<N>;
    const int64_t wgs = pfb_wgs<N>(a);
    if (wgs > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((pfb_fir_fft<N, M, V>), dim3((unsigned)wgs), dim3(P::WG), 0, s, a);
    return hipGetLastError();
}

template <int N, int M>
hipError_t launch_pfb_group_nm(const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((pfb_group<N, M>), dim3((unsigned)grid), dim3(PfbPlan<N>::WG), 0, s, hdr, items);
    return hipGetLastError();
}

template <int N>
hipError_t launch_pfb_group_n(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s)
{
    switch (M) {
    case 1: return launch_pfb_group_nm<N, 1>(hdr, items, grid, s);
    case 2: return launch_pfb_group_nm<N, 2>(hdr, items, grid, s);
    case 3: return launch_pfb_group_nm<N, 3>(hdr, items, grid, s);
    case 4: return launch_pfb_group_nm<N, 4>(hdr, items, grid, s);
    case 5: return launch_pfb_group_nm<N, 5>(hdr, items, grid, s);
    case 6: return launch_pfb_group_nm<N, 6>(hdr, items, grid, s);
    case 7: return launch_pfb_group_nm<N, 7>(hdr, items, grid, s);
    case 8: return launch_pfb_group_nm<N, 8>(hdr, items, grid, s);
    case 9: return launch_pfb_group_nm<N, 9>(hdr, items, grid, s);
    case 10: return launch_pfb_group_nm<N, 10>(hdr, items, grid, s);
    case 11: return launch_pfb_group_nm<N, 11>(hdr, items, grid, s);
    case 12: return launch_pfb_group_nm<N, 12>(hdr, items, grid, s);
    case 13: return launch_pfb_group_nm<N, 13>(hdr, items, grid, s);
    case 14: return launch_pfb_group_nm<N, 14>(hdr, items, grid, s);
    case 15: return launch_pfb_group_nm<N, 15>(hdr, items, grid, s);
    case 16: return launch_pfb_group_nm<N, 16>(hdr, items, grid, s);
    default: return hipErrorInvalidValue;
    }
}

// The grouped kernel for (N, M), as a function pointer (for graph kernel nodes).
template <int N>
const void *pfb_group_fn(int M)
{
    switch (M) {
    case 1: return reinterpret_cast<const void *>(&pfb_group<N, 1>);
    case 2: return reinterpret_cast<const void *>(&pfb_group<N, 2>);
    case 3: return reinterpret_cast<const void *>(&pfb_group<N, 3>);
    case 4: return reinterpret_cast<const void *>(&pfb_group<N, 4>);
    case 5: return reinterpret_cast<const void *>(&pfb_group<N, 5>);
    case 6: return reinterpret_cast<const void *>(&pfb_group<N, 6>);
    case 7: return reinterpret_cast<const void *>(&pfb_group<N, 7>);
    case 8: return reinterpret_cast<const void *>(&pfb_group<N, 8>);
    case 9: return reinterpret_cast<const void *>(&pfb_group<N, 9>);
    case 10: return reinterpret_cast<const void *>(&pfb_group<N, 10>);
    case 11: return reinterpret_cast<const void *>(&pfb_group<N, 11>);
    case 12: return reinterpret_cast<const void *>(&pfb_group<N, 12>);
    case 13: return reinterpret_cast<const void *>(&pfb_group<N, 13>);
    case 14: return reinterpret_cast<const void *>(&pfb_group<N, 14>);
    case 15: return reinterpret_cast<const void *>(&pfb_group<N, 15>);
    case 16: return reinterpret_cast<const void *>(&pfb_group<N, 16>);
    default: return nullptr;
    }
}

// Dispatch over M (1..16) for a fixed N with the default variant.
template <int N, int V>
hipError_t launch_pfb_nv(const PfbLaunch &a, hipStream_t s)
{
    switch (a.M) {
    case 1: return launch_pfb_nmv<N, 1, V>(a, s);
    case 2: return launch_pfb_nmv<N, 2, V>(a, s);
    case 3: return launch_pfb_nmv<N, 3, V>(a, s);
    case 4: return launch_pfb_nmv<N, 4, V>(a, s);
    case 5: return launch_pfb_nmv<N, 5, V>(a, s);
    case 6: return launch_pfb_nmv<N, 6, V>(a, s);
    case 7: return launch_pfb_nmv<N, 7, V>(a, s);
    case 8: return launch_pfb_nmv<N, 8, V>(a, s);
    case 9: return launch_pfb_nmv<N, 9, V>(a, s);
    case 10: return launch_pfb_nmv<N, 10, V>(a, s);
    case 11: return launch_pfb_nmv<N, 11, V>(a, s);
    case 12: return launch_pfb_nmv<N, 12, V>(a, s);
    case 13: return launch_pfb_nmv<N, 13, V>(a, s);
    case 14: return launch_pfb_nmv<N, 14, V>(a, s);
    case 15: return launch_pfb_nmv<N, 15, V>(a, s);
    case 16: return launch_pfb_nmv<N, 16, V>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// Per-N entry points, each defined in its own translation unit.
#define RF_DECL_GROUP(n) hipError_t launch_pfb_group_n##n(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s); \
    const void *pfb_group_fn_n##n(int M);
RF_DECL_GROUP(16) RF_DECL_GROUP(32) RF_DECL_GROUP(64) RF_DECL_GROUP(128) RF_DECL_GROUP(256)
RF_DECL_GROUP(512) RF_DECL_GROUP(1024) RF_DECL_GROUP(2048) RF_DECL_GROUP(4096)
#undef RF_DECL_GROUP
hipError_t launch_pfb_n16(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n32(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n64(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n128(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n256(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n512(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n1024(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n2048(const PfbLaunch &a, hipStream_t s);
hipError_t launch_pfb_n4096(const PfbLaunch &a, hipStream_t s);

}  // namespace rfk
