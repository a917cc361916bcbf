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
//  * A lane group (LG) of L = N/4 threads walks a contiguous run of frames.
//    Thread c of an LG owns the four columns n = c + k*L (k = 0..3), holds their
//    M taps and a window of M+3 blocks of input in registers, and produces four
//    frames per phase.  Its four FIR outputs are exactly the inputs of one
//    radix-4 butterfly of the first Stockham pass (stride N/4, no twiddles),
//    which it computes before writing to LDS.
//  * The remaining passes are radix-16 (radix 8/4/2 for the last one) Stockham
//    passes: a team of N/16 threads owns one frame, every thread holds 16 points
//    per pass.  The last pass writes the natural-order spectrum straight to HBM
//    -- or, when the caller chose a set of channels, back to LDS, from where
//    the frame's team gathers the chosen bins into consecutive columns (same
//    arithmetic, fewer bytes written).
//  * LDS holds the frames of one phase, indexed with one float2 of padding per
//    32 entries (i + (i>>5)): the FIR's radix-4 outputs, four consecutive
//    entries per lane (lanes 32 bytes apart), and the strided stores of the
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

template <int N>
struct PfbPlan {
    static constexpr int L = N / 4;                  // threads per lane group
    static constexpr int WG = L > 256 ? L : 256;     // threads per work-group
    static constexpr int NLG = WG / L;               // lane groups per work-group
    static constexpr int FB = NLG * 4;               // frames per phase buffer
    static constexpr int NT = N / 16;                // FFT team size (threads)
    static constexpr int LDS = FB * N + ((FB * N) >> 5);
    static constexpr bool LG_IN_WAVE = L <= 64;      // FIR and FFT of an LG stay in one wave
    static constexpr bool TEAM_IN_WAVE = NT <= 64;
};

__host__ __device__ constexpr int pass_radix(int N, int NS) { return (N / NS) >= 16 ? 16 : (N / NS); }

// Offset (in float pairs) of the twiddle table of the pass with stride NS.
__host__ __device__ constexpr int tw_offset(int N, int NS)
{
    int off = 0;
    for (int ns = 4; ns < NS;) {
        int R = pass_radix(N, ns);
        off += ns * R;
        ns *= R;
    }
    return off;
}

// Twiddles of R = 16 passes, and of every pass when N <= 2048, are staged in
// LDS; otherwise (the radix-4 last pass of N = 4096) W^k is read once and its
// powers formed by multiplication.
template <int N, int NS>
struct TwPlace {
    static constexpr int R = pass_radix(N, NS);
    static constexpr bool IN_LDS = (R == 16) || (N <= 2048);
};

template <int N>
__host__ __device__ constexpr int lds_tw_count()
{
    int n = 0;
    for (int ns = 4; ns < N;) {
        int R = pass_radix(N, ns);
        if (R == 16 || N <= 2048) n += ns * R;
        ns *= R;
    }
    return n > 0 ? n : 1;
}

__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

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
    return v < vs.H ? vs.hist[v] : vs.in[v - vs.H];
}

__device__ __forceinline__ cf unpack(uint32_t w)
{
    return {(float)(int16_t)(w & 0xffffu), (float)(int16_t)(w >> 16)};
}

// Load four columns c + k*L of virtual block b (samples [bN, bN+N)), resolving
// each against history, new input and end of data.
template <int N>
__device__ __forceinline__ void load_block(const VStream &vs, int64_t vlen, int64_t b, int c,
                                           uint32_t (&w)[4])
{
    constexpr int L = N / 4;
    const int64_t base = b * N;
    if (base + N <= vlen) {
        if (base >= vs.H) {
            const uint32_t *p = vs.in + (base - vs.H) + c;
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = p[k * L];
        } else if (base + N <= vs.H) {
            const uint32_t *p = vs.hist + base + c;
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = p[k * L];
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) w[k] = vload(vs, base + c + k * L);
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
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
__device__ __forceinline__ void fft_pass(cf *lds, int fb, int tl, const cf *twl,
                                         const cf *__restrict__ twg, float *__restrict__ outf,
                                         bool valid, const int32_t *__restrict__ sel)
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
            if constexpr (TwPlace<N, NS>::IN_LDS) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], twl[TOFF + r * NS + k]);
            } else {
                const cf w1 = twg[TOFF + NS + k];
                cf w = w1;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    v[b][r] = cmul(v[b][r], w);
                    if (r + 1 < R) w = cmul(w, w1);
                }
            }
        }
        dft<R>(v[b]);
        const int idxD = (j / NS) * NS * R + k;
        if constexpr (LAST && !SEL) {
            if (valid) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    f2v o = {v[b][r].x, v[b][r].y};
                    f2v *dst = (f2v *)(outf + 2 * (idxD + r * NS));
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
__device__ __forceinline__ void fft_passes(cf *lds, int fb, int tl, const cf *twl,
                                           const cf *__restrict__ twg, float *__restrict__ outf,
                                           bool valid, const int32_t *__restrict__ sel, int nsel)
{
    if constexpr (NS < N) {
        constexpr int R = pass_radix(N, NS);
        fft_pass<N, R, NS, NS * R == N, NT_STORE, SEL || STAGED>(lds, fb, tl, twl, twg, outf, valid, sel);
        fft_passes<N, NS * R, NT_STORE, SEL, STAGED>(lds, fb, tl, twl, twg, outf, valid, sel, nsel);
    } else if constexpr (SEL) {
        // the spectrum is in LDS: the team gathers the chosen bins into
        // consecutive columns (sel = the bins, in output order)
        group_sync<!PfbPlan<N>::TEAM_IN_WAVE>();
        if (valid) {
            for (int c = tl; c < nsel; c += PfbPlan<N>::NT) {
                const cf x = lds[lpad(fb + sel[c])];
                f2v o = {x.x, x.y};
                f2v *dst = (f2v *)(outf + 2 * c);
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

template <int N, int M>
struct FirState {
    static constexpr bool PACKED = (M > 8) || (N >= 4096);
    static constexpr int W = M + 3;   // window blocks fp .. fp+M+2
    float hr[M][4];
    WinT<PACKED> xw[W][4];
};

// FIR of the phase's four frames, first radix-4 pass, store to LDS.
template <int N, int M>
__device__ __forceinline__ void fir_phase(const FirState<N, M> &st, cf *lds, int g, int c)
{
#pragma unroll
    for (int qf = 0; qf < 4; ++qf) {
        cf v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            cf s = {0.f, 0.f};
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const cf x = st.xw[qf + m][k].get();
                s.x = __builtin_fmaf(st.hr[m][k], x.x, s.x);
                s.y = __builtin_fmaf(st.hr[m][k], x.y, s.y);
            }
            v[k] = s;
        }
        dft4(v[0], v[1], v[2], v[3]);
        // entries 4c .. 4c+3 never straddle a padding point (every 32)
        cf *dst = lds + lpad((g * 4 + qf) * N + 4 * c);
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[r] = v[r];
    }
}

template <int N, int M>
__device__ __forceinline__ void shift_window(FirState<N, M> &st, const uint32_t (&pre)[4][4])
{
    constexpr int W = FirState<N, M>::W;
#pragma unroll
    for (int i = 0; i + 4 < W; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) st.xw[i][k] = st.xw[i + 4][k];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 4; ++k) st.xw[W - 4 + i][k].set(pre[i][k]);
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
                f2v *dst = (f2v *)(out + 2 * (fg * N + e));
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

// LDS of the PFB body, sized for its plan and variant.
template <int N, int V>
struct PfbShared {
    cf frames[PfbVariant<N, V>::NBUF * PfbPlan<N>::LDS];
    cf tw[lds_tw_count<N>()];
};

// The whole PFB computation of one logical work-group `lwg` of `G` for the
// call described by `a`.  Shared by the single-stream kernel and the grouped
// multi-stream kernel, so a stream's frames are computed by the same
// instructions either way.  OPAQUE (callers that run the body in a loop):
// the thread index is hidden from the optimiser, so each run's per-thread
// addresses are computed in it instead of being kept live across runs.
template <int N, int M, int V, bool OPAQUE = false>
__device__ __forceinline__ void pfb_body(const PfbLaunch &a, int lwg, int G, PfbShared<N, V> &sh)
{
    using P = PfbPlan<N>;
    using VV = PfbVariant<N, V>;
    constexpr int L = P::L;
    constexpr int W = FirState<N, M>::W;
    constexpr int TWL = lds_tw_count<N>();
    // one barrier per phase when double buffered, else two
    constexpr bool SYNC2 = !P::LG_IN_WAVE && !VV::DBUF;
    cf *lds_all = sh.frames;
    cf *twl = sh.tw;

    int tid = threadIdx.x;
    if constexpr (OPAQUE) {
        asm volatile("" : "+v"(tid));
        __builtin_assume(tid >= 0 && tid < P::WG);
    }
    const cf *twg = reinterpret_cast<const cf *>(a.tw);
    for (int i = tid; i < TWL; i += P::WG) twl[i] = twg[i];

    const VStream vs = a.vs;
    const int64_t vlen = vs.H + vs.n;
    const int64_t F = a.F;
    const int RL = a.run_len;
    const int nph = RL >> 2;
    // output row length: all N bins, or the chosen channels (variant bit 8:
    // a.sel lists the bins in output order; compiled only into that variant)
    constexpr bool SEL = (V & 8) != 0;
    constexpr bool STAGE = PfbStage<N>::ON && !SEL;
    const int32_t *sel = SEL ? a.sel : nullptr;
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
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int k = 0; k < 4; ++k) st.hr[m][k] = a.taps[m * N + c + k * L];

    // FFT team of this thread (may belong to another lane group for N >= 512)
    const int slot = tid / P::NT;
    const int tl = tid - slot * P::NT;
    const int lg2 = slot >> 2, q2 = slot & 3;
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
            const uint32_t *base = vs.in + (f0 * N - vs.H) + c;
            const int64_t b0 = back ? 4 * (int64_t)(nph - 1) : 0;   // first window block
#pragma unroll
            for (int i = 0; i < W; ++i)
#pragma unroll
                for (int k = 0; k < 4; ++k) st.xw[i][k].set(base[(b0 + i) * N + k * L]);
#pragma unroll 1
            for (int it = 0; it < nph; ++it) {
                const int ph = back ? nph - 1 - it : it;
                cf *lds = lds_all + (VV::DBUF ? (it & 1) * P::LDS : 0);
                uint32_t pre[4][4];
                const bool more = it + 1 < nph;
                if (more) {
                    const uint32_t *p = base + (int64_t)(back ? 4 * ph - 4 : 4 * ph + W) * N;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int k = 0; k < 4; ++k) pre[i][k] = p[i * N + k * L];
                }
                fir_phase<N, M>(st, lds, g, c);
                group_sync<!P::LG_IN_WAVE>();
                fft_passes<N, 4, VV::NT_STORE, SEL, STAGE>(lds, slot * N, tl, twl, twg,
                                                      a.out + 2 * (f0t + 4 * ph + q2) * ldo, true, sel, a.nsel);
                if constexpr (STAGE) {
                    wave_fence();
                    staged_copy<N, VV::NT_STORE>(lds, a.out, (int64_t)lwg * P::NLG, RL, ph, F);
                }
                if constexpr (SYNC2) group_sync<true>();
                else wave_fence();
                if (more) {
                    if (back) {
#pragma unroll
                        for (int i = W - 1; i >= 4; --i)
#pragma unroll
                            for (int k = 0; k < 4; ++k) st.xw[i][k] = st.xw[i - 4][k];
#pragma unroll
                        for (int i = 0; i < 4; ++i)
#pragma unroll
                            for (int k = 0; k < 4; ++k) st.xw[i][k].set(pre[i][k]);
                    } else {
                        shift_window<N, M>(st, pre);
                    }
                }
            }
        }
    }
    if (fast && (V & 16) == 0) {
        // block b of this lane group starts at in + (f0 + b)*N - H
        const uint32_t *base = vs.in + (f0 * N - vs.H) + c;
#pragma unroll
        for (int i = 0; i < W; ++i)
#pragma unroll
            for (int k = 0; k < 4; ++k) st.xw[i][k].set(base[i * N + k * L]);
        auto phase = [&](int ph) __attribute__((always_inline)) {
            cf *lds = lds_all + (VV::DBUF ? (ph & 1) * P::LDS : 0);
            uint32_t pre[4][4];
            const bool more = ph + 1 < nph;
            if (more) {
                const uint32_t *p = base + (int64_t)(4 * ph + W) * N;
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int k = 0; k < 4; ++k) pre[i][k] = p[i * N + k * L];
            }
            fir_phase<N, M>(st, lds, g, c);
            group_sync<!P::LG_IN_WAVE>();
            fft_passes<N, 4, VV::NT_STORE, SEL, STAGE>(lds, slot * N, tl, twl, twg,
                                                  a.out + 2 * (f0t + 4 * ph + q2) * ldo, true, sel, a.nsel);
            if constexpr (STAGE) {
                wave_fence();
                staged_copy<N, VV::NT_STORE>(lds, a.out, (int64_t)lwg * P::NLG, RL, ph, F);
            }
            if constexpr (SYNC2) group_sync<true>();
            else wave_fence();
            if (more) shift_window<N, M>(st, pre);
        };
        // Three phases bring in 12 blocks; for M <= 9 that is more than the
        // window holds, so in a group of three no window value survives to the
        // loop edge and the window needs no register rotation there (a move
        // per value).
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
            uint32_t w[4];
            load_block<N>(vs, vlen, f0 + i, c, w);
#pragma unroll
            for (int k = 0; k < 4; ++k) st.xw[i][k].set(w[k]);
        }
        for (int ph = 0; ph < nph; ++ph) {
            cf *lds = lds_all + (VV::DBUF ? (ph & 1) * P::LDS : 0);
            const int64_t fp = f0 + 4 * ph;
            uint32_t pre[4][4];
            const bool more = (ph + 1 < nph) && (fp + 4 < F);
            if (more) {
#pragma unroll
                for (int i = 0; i < 4; ++i) load_block<N>(vs, vlen, fp + W + i, c, pre[i]);
            }
            if (fp < F) fir_phase<N, M>(st, lds, g, c);
            group_sync<!P::LG_IN_WAVE>();
            {
                const int64_t f = f0t + 4 * ph + q2;
                const bool valid = f < f1t;
                fft_passes<N, 4, VV::NT_STORE, SEL, STAGE>(lds, slot * N, tl, twl, twg,
                                                      a.out + 2 * (valid ? f : 0) * ldo, valid, sel, a.nsel);
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
        a.hist_out[i] = vload(vs, a.keep_from + i);
}

template <int N, int M, int V>
__global__ void __launch_bounds__(PfbPlan<N>::WG) __attribute__((amdgpu_waves_per_eu(M <= 8 ? 2 : 1))) pfb_fir_fft(PfbLaunch a)
{
    __shared__ PfbShared<N, V> sh;
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
__global__ void __launch_bounds__(PfbPlan<N>::WG) pfb_group(const GroupHeader *hdr, const PfbItem *items)
{
    __shared__ PfbShared<N, 0> sh;
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
#define RF_DECL_GROUP(n) hipError_t launch_pfb_group_n##n(int M, const GroupHeader *hdr, const PfbItem *items, int grid, hipStream_t s);
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
