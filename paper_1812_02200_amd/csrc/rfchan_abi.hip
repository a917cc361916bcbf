// rfchan_abi.hip -- C ABI, handle state and stream bookkeeping (host side).
//
// Host-side counting decides, before any kernel runs, how many frames / outputs
// a call emits and which samples must be retained; the kernels receive these as
// plain arguments.  Retained samples live in two device buffers used in turn
// (the kernel reads one and writes the other), so a process call never waits
// for the device and never allocates.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <sys/stat.h>

#include <mutex>
#include <new>
#include <string>

#include "../../include/rfchan.h"
#include "rf_handles.hpp"
#include "rf_internal.hpp"

#define RF_VERSION (0 * 10000 + 1 * 100 + 0)

namespace {

thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(RF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                    \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) {                \
            (void)hipGetLastError();           \
            return hip_fail(e_, what);         \
        }                                      \
    } while (0)

// Keeps the caller's current device while a handle's device is made current.
struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    hipError_t err = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        err = hipGetDevice(&prev);
        if (err == hipSuccess && prev != dev) {
            err = hipSetDevice(dev);
            changed = (err == hipSuccess);
        }
    }
    ~DeviceGuard()
    {
        if (changed) (void)hipSetDevice(prev);
    }
};

// Order this call after the previous call on the same handle when the two
// name different streams.
struct StreamOrder {
    hipStream_t last = nullptr;
    bool has_last = false;
    hipEvent_t ev = nullptr;

    int before(hipStream_t s)
    {
        if (has_last && last != s) {
            HIP_TRY(hipEventRecord(ev, last), "hipEventRecord");
            HIP_TRY(hipStreamWaitEvent(s, ev, 0), "hipStreamWaitEvent");
        }
        return RF_OK;
    }
    void after(hipStream_t s)
    {
        last = s;
        has_last = true;
    }
    int sync()
    {
        if (has_last) HIP_TRY(hipStreamSynchronize(last), "hipStreamSynchronize");
        return RF_OK;
    }
};

template <typename T>
int dev_alloc(T **p, size_t count, const char *what)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? RF_ENOMEM : RF_EDEVICE, "hipMalloc(%s): %s", what,
                    hipGetErrorString(e));
    }
    return RF_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

int device_cus(int dev)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus;
}

}  // namespace

// ====================================================================== PFB

struct rf_pfb {
    int N = 0, M = 0, mode = 0;
    uint64_t max_samples = 0;
    int device = 0;
    float *d_taps = nullptr;
    float *d_tw = nullptr;
    uint32_t *d_hist[2] = {nullptr, nullptr};
    int cur = 0;
    uint64_t S = 0;        // samples received
    uint64_t frames = 0;   // frames emitted
    int64_t H = 0;         // retained samples (virtual stream starts at frames*N)
    int run_len = 0;       // 0: heuristic
    int variant = 0;       // kernel variant bits
    int32_t *d_sel = nullptr;   // [N] capacity: chosen bins in output order
    int nsel = 0;               // 0: every bin
    // large or non-power-of-two N: separate fold and four-step FFT passes
    bool large = false;
    rfk::LargePlan lplan;
    rfk::LargeBuffers lbuf;
    float *d_ltab = nullptr;
    rfk::cf *d_lv = nullptr, *d_ly = nullptr;
    StreamOrder order;
};

namespace {

struct PfbStateBlob {
    uint32_t magic;
    uint32_t version;
    int32_t N, M;
    uint64_t S, frames;
    int64_t H;
};
constexpr uint32_t kPfbMagic = 0x42504652u;  // "RFPB"

void pfb_free(rf_pfb *p)
{
    if (!p) return;
    (void)hipFree(p->d_taps);
    (void)hipFree(p->d_tw);
    (void)hipFree(p->d_hist[0]);
    (void)hipFree(p->d_hist[1]);
    (void)hipFree(p->d_sel);
    (void)hipFree(p->d_ltab);
    (void)hipFree(p->d_lv);
    (void)hipFree(p->d_ly);
    if (p->order.ev) (void)hipEventDestroy(p->order.ev);
    delete p;
}

uint64_t pfb_count(const rf_pfb *p, uint64_t n)
{
    const uint64_t vlen = (uint64_t)p->H + n;
    const uint64_t span = (uint64_t)p->N * p->M;
    return vlen >= span ? (vlen - span) / p->N + 1 : 0;
}

}  // namespace

namespace rfi {

int set_error(int status, const char *msg) { return fail(status, "%s", msg); }

int pfb_prepare(rf_pfb *p, const int16_t *iq_dev, uint64_t nsamples, float *out_dev, uint64_t out_cap_frames,
                rfk::PfbLaunch *a, uint64_t *frames)
{
    if (!p) return fail(RF_EINVAL, "pfb_process: handle is NULL");
    if (nsamples > p->max_samples)
        return fail(RF_EINVAL, "pfb_process: nsamples=%llu exceeds max_samples_per_call=%llu",
                    (unsigned long long)nsamples, (unsigned long long)p->max_samples);
    if (nsamples > 0 && (!iq_dev || !aligned(iq_dev, 4)))
        return fail(RF_EINVAL, "pfb_process: iq_dev must be a non-NULL 4-byte aligned device pointer");
    const uint64_t F = pfb_count(p, nsamples);
    if (F > out_cap_frames)
        return fail(RF_ECAPACITY, "pfb_process: %llu frames need more than out_cap_frames=%llu",
                    (unsigned long long)F, (unsigned long long)out_cap_frames);
    if (F > 0 && (!out_dev || !aligned(out_dev, 8)))
        return fail(RF_EINVAL, "pfb_process: out_dev must be a non-NULL 8-byte aligned device pointer");
    const int64_t vlen = p->H + (int64_t)nsamples;
    a->vs.hist = p->d_hist[p->cur];
    a->vs.in = reinterpret_cast<const uint32_t *>(iq_dev);
    a->vs.H = p->H;
    a->vs.n = (int64_t)nsamples;
    a->hist_out = p->d_hist[p->cur ^ 1];
    a->keep_from = (int64_t)F * p->N;
    a->keep_len = vlen - a->keep_from;
    a->out = out_dev;
    a->taps = p->d_taps;
    a->tw = p->d_tw;
    a->F = (int64_t)F;
    a->run_len = p->run_len > 0 ? p->run_len : rfk::pfb_default_run_len(p->N, p->M, (int64_t)F);
    a->N = p->N;
    a->M = p->M;
    a->variant = p->variant;
    a->sel = p->nsel > 0 ? p->d_sel : nullptr;
    a->nsel = p->nsel;
    *frames = F;
    return RF_OK;
}

void pfb_commit(rf_pfb *p, const rfk::PfbLaunch &a, uint64_t nsamples, uint64_t F, hipStream_t s)
{
    p->order.after(s);
    p->cur ^= 1;
    p->H = a.keep_len;
    p->S += nsamples;
    p->frames += F;
}

int pfb_device(const rf_pfb *p) { return p->device; }
int pfb_mode(const rf_pfb *p) { return p->mode; }
size_t pfb_footprint(int N, int M, int mode)
{
    const size_t span = (size_t)N * M;
    const size_t tw = mode == RF_DFT_FFT_F32 ? (size_t)rfk::pfb_twiddle_count(N) * 8
                                             : (size_t)rfk::pfb_mfma_table_floats() * 4;
    const size_t taps = (rfk::pfb_fir_radix(N) == 8 && mode == RF_DFT_FFT_F32 ? 2 : 1) * span * 4;
    return taps + tw + 2 * span * 4 /* history */;
}

}  // namespace rfi

extern "C" {

const char *rf_strerror(int status)
{
    switch (status) {
    case RF_OK: return "ok";
    case RF_EINVAL: return "invalid argument";
    case RF_ENOMEM: return "out of memory";
    case RF_EDEVICE: return "HIP runtime error";
    case RF_ECAPACITY: return "output capacity too small";
    case RF_EAGAIN: return "resource busy, try again";
    case RF_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

const char *rf_last_error(void) { return g_last_error.c_str(); }

int rf_version(void) { return RF_VERSION; }

int pfb_create(rf_pfb_t *out, int32_t nchan, int32_t ntaps, const float *proto, int32_t dft_mode,
               uint64_t max_samples_per_call)
{
    if (!out) return fail(RF_EINVAL, "pfb_create: out is NULL");
    *out = nullptr;
    const bool fused = nchan >= 16 && nchan <= 4096 && !(nchan & (nchan - 1));
    if (!fused && !rfk::large_supported(nchan))
        return fail(RF_EINVAL,
                    "pfb_create: nchan=%d must be a power of two in [16, 4096] or a product of "
                    "powers of 2, 3 and 5 in [16, 2^24] splitting into two factors <= 4096", nchan);
    if (!fused && dft_mode != RF_DFT_FFT_F32)
        return fail(RF_EUNSUPPORTED, "pfb_create: large or non-power-of-two nchan needs the FP32 FFT mode");
    if (ntaps < 1 || ntaps > 16) return fail(RF_EINVAL, "pfb_create: ntaps=%d must be in [1, 16]", ntaps);
    if (!proto) return fail(RF_EINVAL, "pfb_create: proto is NULL");
    if (max_samples_per_call < 1 || max_samples_per_call > (1ull << 40))
        return fail(RF_EINVAL, "pfb_create: max_samples_per_call out of range");
    if (dft_mode != RF_DFT_FFT_F32 && dft_mode != RF_DFT_MFMA_F16X2 && dft_mode != RF_DFT_MFMA_BF16X2)
        return fail(RF_EINVAL, "pfb_create: unknown dft_mode %d", dft_mode);
    if (dft_mode != RF_DFT_FFT_F32 && (!fused || nchan > 256))
        return fail(RF_EUNSUPPORTED, "pfb_create: the MFMA DFT modes support nchan = 16, 32, 64, 128, 256");
    for (int i = 0; i < nchan * ntaps; ++i)
        if (!isfinite(proto[i])) return fail(RF_EINVAL, "pfb_create: proto[%d] is not finite", i);
    // MFMA modes: taps scaled by 2^e (exact) so that no half-precision operand
    // can overflow; the kernel scales its outputs back by 2^-e
    int mfma_exp = 0;
    if (dft_mode != RF_DFT_FFT_F32 && !rfk::pfb_mfma_scale_exponent(proto, nchan, ntaps, &mfma_exp))
        return fail(RF_EUNSUPPORTED, "pfb_create: taps too large for the half-precision MFMA DFT");

    rf_pfb *p = new (std::nothrow) rf_pfb;
    if (!p) return fail(RF_ENOMEM, "pfb_create: host allocation");
    p->N = nchan;
    p->M = ntaps;
    p->mode = dft_mode;
    p->max_samples = max_samples_per_call;
    int rc = RF_OK;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        pfb_free(p);
        return hip_fail(e, "hipGetDevice");
    }
    const size_t span = (size_t)nchan * ntaps;
    if (!fused) {
        p->large = true;
        rfk::large_plan(nchan, &p->lplan);
        const size_t nt = rfk::large_table_floats(p->lplan);
        const size_t fcap = max_samples_per_call / (uint64_t)nchan + 2;   // frames one call can emit
        float *tab = (float *)malloc(sizeof(float) * nt);
        if (!tab) {
            pfb_free(p);
            return fail(RF_ENOMEM, "pfb_create: host allocation");
        }
        rfk::large_table_fill(p->lplan, tab);
        if ((rc = dev_alloc(&p->d_taps, span, "taps")) || (rc = dev_alloc(&p->d_ltab, nt, "twiddles")) ||
            (rc = dev_alloc(&p->d_hist[0], span, "history")) || (rc = dev_alloc(&p->d_hist[1], span, "history")) ||
            (rc = dev_alloc(&p->d_lv, fcap * nchan, "fold scratch")) ||
            (rc = dev_alloc(&p->d_ly, fcap * nchan, "FFT scratch"))) {
            free(tab);
            pfb_free(p);
            return rc;
        }
        e = hipMemcpy(p->d_taps, proto, span * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->d_ltab, tab, sizeof(float) * nt, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->order.ev, hipEventDisableTiming);
        free(tab);
        if (e != hipSuccess) {
            pfb_free(p);
            return hip_fail(e, "pfb_create");
        }
        p->lbuf.v = p->d_lv;
        p->lbuf.y = p->d_ly;
        p->lbuf.tables = p->d_ltab;
        *out = p;
        return RF_OK;
    }
    // FFT: pass twiddle tables (float pairs); MFMA: DFT16 block matrix + W256 twiddles
    const int ntw = dft_mode == RF_DFT_FFT_F32 ? rfk::pfb_twiddle_count(nchan)
                                               : (rfk::pfb_mfma_table_floats() + 1) / 2;
    float *tw = (float *)malloc(sizeof(float) * 2 * ntw);
    if (!tw) {
        pfb_free(p);
        return fail(RF_ENOMEM, "pfb_create: host allocation");
    }
    // Eight columns per thread (N = 4096): the natural layout is followed by a
    // copy [m][q][c][k] = h[m N + c + (4q + k) N/8] that the kernel reads as
    // 16-byte parts, consecutive threads at consecutive parts
    const int fir_c = rfk::pfb_fir_radix(nchan);
    const size_t ntaps_dev = fir_c == 8 && dft_mode == RF_DFT_FFT_F32 ? 2 * span : span;
    float *taps = (float *)malloc(sizeof(float) * ntaps_dev);
    if (!taps) {
        free(tw);
        pfb_free(p);
        return fail(RF_ENOMEM, "pfb_create: host allocation");
    }
    if (dft_mode == RF_DFT_FFT_F32) {
        rfk::pfb_twiddle_fill(nchan, tw);
        memcpy(taps, proto, sizeof(float) * span);
        if (ntaps_dev > span) {
            const int L = nchan / fir_c;
            for (int m = 0; m < ntaps; ++m)
                for (int q = 0; q < fir_c / 4; ++q)
                    for (int c = 0; c < L; ++c)
                        for (int k = 0; k < 4; ++k)
                            taps[span + (((size_t)m * (fir_c / 4) + q) * L + c) * 4 + k] =
                                proto[(size_t)m * nchan + c + (4 * q + k) * L];
        }
    } else {
        rfk::pfb_mfma_table_fill(nchan, mfma_exp, tw);
        for (size_t i = 0; i < span; ++i) taps[i] = ldexpf(proto[i], mfma_exp);
    }
    if ((rc = dev_alloc(&p->d_taps, ntaps_dev, "taps")) || (rc = dev_alloc(&p->d_tw, 2 * (size_t)ntw, "twiddles")) ||
        (rc = dev_alloc(&p->d_hist[0], span, "history")) || (rc = dev_alloc(&p->d_hist[1], span, "history"))) {
        free(tw);
        free(taps);
        pfb_free(p);
        return rc;
    }
    e = hipMemcpy(p->d_taps, taps, ntaps_dev * sizeof(float), hipMemcpyHostToDevice);
    free(taps);
    if (e == hipSuccess) e = hipMemcpy(p->d_tw, tw, sizeof(float) * 2 * ntw, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->order.ev, hipEventDisableTiming);
    free(tw);
    if (e != hipSuccess) {
        pfb_free(p);
        return hip_fail(e, "pfb_create");
    }
    const char *rl = getenv("RFCHAN_PFB_RUN_LEN");
    if (rl) {
        int v = atoi(rl);
        if (v >= 4 && v % 4 == 0) p->run_len = v;
    }
    const char *vr = getenv("RFCHAN_PFB_VARIANT");
    if (vr) p->variant = atoi(vr);
    *out = p;
    return RF_OK;
}

int pfb_set_channels(rf_pfb_t p, const int32_t *channels, int32_t nsel)
{
    if (!p) return fail(RF_EINVAL, "pfb_set_channels: handle is NULL");
    if (nsel < 0 || nsel > p->N) return fail(RF_EINVAL, "pfb_set_channels: nsel=%d must be in [0, N]", nsel);
    if (nsel > 0 && !channels) return fail(RF_EINVAL, "pfb_set_channels: channels is NULL");
    if (nsel > 0 && (p->mode != RF_DFT_FFT_F32 || p->large))
        return fail(RF_EUNSUPPORTED,
                    "pfb_set_channels: chosen channels need the FP32 FFT mode and a power-of-two N <= 4096");
    int32_t *map = (int32_t *)malloc(sizeof(int32_t) * p->N);
    if (!map) return fail(RF_ENOMEM, "pfb_set_channels: host allocation");
    for (int k = 0; k < p->N; ++k) map[k] = -1;
    for (int c = 0; c < nsel; ++c) {
        const int32_t k = channels[c];
        if (k < 0 || k >= p->N || map[k] >= 0) {
            free(map);
            return fail(RF_EINVAL, "pfb_set_channels: channel %d is out of range or repeated", (int)k);
        }
        map[k] = c;
    }
    DeviceGuard dg(p->device);
    if (dg.err != hipSuccess) {
        free(map);
        return hip_fail(dg.err, "hipSetDevice");
    }
    int rc = p->order.sync();
    if (rc == RF_OK && nsel > 0 && !p->d_sel) rc = dev_alloc(&p->d_sel, (size_t)p->N, "channel map");
    if (rc == RF_OK && nsel > 0) {
        const hipError_t e = hipMemcpy(p->d_sel, channels, sizeof(int32_t) * nsel, hipMemcpyHostToDevice);
        if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy(channel map)");
    }
    free(map);
    if (rc) return rc;
    p->nsel = nsel;
    return RF_OK;
}

uint64_t pfb_frames_for(rf_pfb_t pfb, uint64_t nsamples)
{
    if (!pfb) return 0;
    return pfb_count(pfb, nsamples);
}

int pfb_process(rf_pfb_t p, const int16_t *iq_dev, uint64_t nsamples, float *out_dev, uint64_t out_cap_frames,
                uint64_t *frames_out, void *hip_stream)
{
    if (frames_out) *frames_out = 0;
    rfk::PfbLaunch a;
    uint64_t F = 0;
    int rc = rfi::pfb_prepare(p, iq_dev, nsamples, out_dev, out_cap_frames, &a, &F);
    if (rc || nsamples == 0) return rc;

    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    rc = p->order.before(s);
    if (rc) return rc;
    if (p->large)
        HIP_TRY(rfk::launch_pfb_large(a, p->lplan, p->lbuf, s), "pfb large-N launch");
    else if (p->mode == RF_DFT_FFT_F32)
        HIP_TRY(rfk::launch_pfb(a, s), "pfb kernel launch");
    else
        HIP_TRY(rfk::launch_pfb_mfma(a, p->mode == RF_DFT_MFMA_BF16X2 ? rfk::RF_PREC_BF16 : rfk::RF_PREC_F16, s),
                "pfb mfma kernel launch");
    rfi::pfb_commit(p, a, nsamples, F, s);
    if (frames_out) *frames_out = F;
    return RF_OK;
}

}  // extern "C"

// ------------------------------------------- process call without allocation
//
// The large-N path's kernels work through two scratch arrays (the folded
// frames and the first FFT step's output).  pfb_process_static takes them from
// this file-scope device array instead of the handle's own buffers, so a
// caller that cannot allocate (code under graph capture, serving loops) still
// has a call whose scratch memory is fixed in advance.  Each GPU holds its own
// copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the device that is current.
namespace {

constexpr size_t kStaticScratchBytes = 64ull << 20;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on device `dev` (the current device), looked
// up once per device.
int static_scratch(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(RF_EUNSUPPORTED, "pfb_process_static: device index %d", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(RF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return RF_OK;
}

}  // namespace

extern "C" {

int pfb_process_static(rf_pfb_t p, const int16_t *iq_dev, uint64_t nsamples, float *out_dev,
                       uint64_t out_cap_frames, uint64_t *frames_out, void *hip_stream)
{
    if (frames_out) *frames_out = 0;
    rfk::PfbLaunch a;
    uint64_t F = 0;
    int rc = rfi::pfb_prepare(p, iq_dev, nsamples, out_dev, out_cap_frames, &a, &F);
    if (rc || nsamples == 0) return rc;
    size_t vbytes = 0;
    if (p->large) {
        // folded frames, then (two-step plans) the first step's output
        vbytes = ((size_t)F * (size_t)p->N * sizeof(rfk::cf) + 255) & ~(size_t)255;
        const size_t need = p->lplan.N2 > 1 ? 2 * vbytes : vbytes;
        if (need > kStaticScratchBytes)
            return fail(RF_EINVAL,
                        "pfb_process_static: %llu frames of %d channels need %zu bytes of scratch, more than "
                        "the %zu-byte static scratch (use pfb_process, or fewer samples per call)",
                        (unsigned long long)F, p->N, need, kStaticScratchBytes);
    }
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    rfk::LargeBuffers lb = p->lbuf;
    if (p->large) {
        void *base = nullptr;
        if ((rc = static_scratch(p->device, &base))) return rc;
        lb.v = reinterpret_cast<rfk::cf *>(base);
        lb.y = reinterpret_cast<rfk::cf *>(static_cast<unsigned char *>(base) + vbytes);
    }
    rc = p->order.before(s);
    if (rc) return rc;
    if (p->large)
        HIP_TRY(rfk::launch_pfb_large(a, p->lplan, lb, s), "pfb large-N launch");
    else if (p->mode == RF_DFT_FFT_F32)
        HIP_TRY(rfk::launch_pfb(a, s), "pfb kernel launch");
    else
        HIP_TRY(rfk::launch_pfb_mfma(a, p->mode == RF_DFT_MFMA_BF16X2 ? rfk::RF_PREC_BF16 : rfk::RF_PREC_F16, s),
                "pfb mfma kernel launch");
    rfi::pfb_commit(p, a, nsamples, F, s);
    if (frames_out) *frames_out = F;
    return RF_OK;
}

int pfb_counters(rf_pfb_t p, uint64_t *samples_in, uint64_t *frames_out, uint64_t *history_samples)
{
    if (!p) return fail(RF_EINVAL, "pfb_counters: handle is NULL");
    if (samples_in) *samples_in = p->S;
    if (frames_out) *frames_out = p->frames;
    if (history_samples) *history_samples = (uint64_t)p->H;
    return RF_OK;
}

int pfb_get_state(rf_pfb_t p, void *blob, size_t *size)
{
    if (!p || !size) return fail(RF_EINVAL, "pfb_get_state: NULL argument");
    const size_t need = sizeof(PfbStateBlob) + (size_t)p->H * 4;
    if (!blob) {
        *size = need;
        return RF_OK;
    }
    if (*size < need) {
        *size = need;
        return fail(RF_ECAPACITY, "pfb_get_state: blob needs %zu bytes", need);
    }
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    PfbStateBlob h = {kPfbMagic, 1, p->N, p->M, p->S, p->frames, p->H};
    memcpy(blob, &h, sizeof h);
    if (p->H > 0)
        HIP_TRY(hipMemcpy((char *)blob + sizeof h, p->d_hist[p->cur], (size_t)p->H * 4, hipMemcpyDeviceToHost),
                "hipMemcpy(state)");
    *size = need;
    return RF_OK;
}

int pfb_set_state(rf_pfb_t p, const void *blob, size_t size)
{
    if (!p || !blob) return fail(RF_EINVAL, "pfb_set_state: NULL argument");
    PfbStateBlob h;
    if (size < sizeof h) return fail(RF_EINVAL, "pfb_set_state: blob too small");
    memcpy(&h, blob, sizeof h);
    if (h.magic != kPfbMagic || h.version != 1) return fail(RF_EINVAL, "pfb_set_state: not a PFB state blob");
    if (h.N != p->N || h.M != p->M) return fail(RF_EINVAL, "pfb_set_state: blob is for N=%d M=%d", h.N, h.M);
    if (h.H < 0 || h.H >= (int64_t)p->N * p->M || size < sizeof h + (size_t)h.H * 4)
        return fail(RF_EINVAL, "pfb_set_state: inconsistent history length");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    if (h.H > 0)
        HIP_TRY(hipMemcpy(p->d_hist[p->cur], (const char *)blob + sizeof h, (size_t)h.H * 4, hipMemcpyHostToDevice),
                "hipMemcpy(state)");
    p->S = h.S;
    p->frames = h.frames;
    p->H = h.H;
    return RF_OK;
}

int pfb_reset(rf_pfb_t p)
{
    if (!p) return fail(RF_EINVAL, "pfb_reset: handle is NULL");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    p->S = 0;
    p->frames = 0;
    p->H = 0;
    return RF_OK;
}

int pfb_destroy(rf_pfb_t p)
{
    if (!p) return RF_OK;
    int rc = RF_OK;
    {
        DeviceGuard dg(p->device);
        if (dg.err == hipSuccess) rc = p->order.sync();
        pfb_free(p);
    }
    return rc;
}

}  // extern "C"

// ====================================================================== DDC

struct rf_ddc {
    int ntones = 0, T = 0, D = 0;
    uint64_t max_samples = 0;
    int device = 0;
    int cus = 256;
    uint64_t *d_inc = nullptr, *d_phi0 = nullptr, *d_phase = nullptr;
    uint64_t *d_chirp = nullptr;   // phase second differences (chirped tones) or null
    float *d_wrev = nullptr, *d_tab = nullptr;
    uint32_t *d_hist[2] = {nullptr, nullptr};
    int cur = 0;
    uint64_t S = 0;       // samples received
    uint64_t nnext = 0;   // outputs emitted (absolute index of the next output)
    int64_t H = 0;        // retained samples, absolute [S-H, S) == [nnext*D, S)
    uint64_t skip = 0;    // samples of future input before nnext*D (only when D > T)
    uint64_t *h_inc = nullptr, *h_phi0 = nullptr, *h_chirp = nullptr;
    float *h_taps = nullptr;
    int grid = 0;
    StreamOrder order;
};

namespace {

struct DdcStateBlob {
    uint32_t magic;
    uint32_t version;
    int32_t ntones, T, D, pad;
    uint64_t S, nnext, skip;
    int64_t H;
    uint64_t fingerprint;
};
constexpr uint32_t kDdcMagic = 0x43444652u;  // "RFDC"

void ddc_free(rf_ddc *p)
{
    if (!p) return;
    (void)hipFree(p->d_inc);
    (void)hipFree(p->d_phi0);
    (void)hipFree(p->d_phase);
    (void)hipFree(p->d_chirp);
    (void)hipFree(p->d_wrev);
    (void)hipFree(p->d_tab);
    (void)hipFree(p->d_hist[0]);
    (void)hipFree(p->d_hist[1]);
    if (p->order.ev) (void)hipEventDestroy(p->order.ev);
    free(p->h_inc);
    free(p->h_phi0);
    free(p->h_chirp);
    free(p->h_taps);
    delete p;
}

// FNV-1a over the configuration, so a state blob only restores onto the same bank.
uint64_t ddc_fingerprint(const rf_ddc *p)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *d, size_t n) {
        const unsigned char *c = (const unsigned char *)d;
        for (size_t i = 0; i < n; ++i) {
            h ^= c[i];
            h *= 1099511628211ull;
        }
    };
    mix(&p->ntones, sizeof p->ntones);
    mix(&p->T, sizeof p->T);
    mix(&p->D, sizeof p->D);
    mix(p->h_inc, sizeof(uint64_t) * p->ntones);
    mix(p->h_phi0, sizeof(uint64_t) * p->ntones);
    mix(p->h_taps, sizeof(float) * p->T);
    if (p->h_chirp) mix(p->h_chirp, sizeof(uint64_t) * p->ntones);
    return h;
}

// m(m-1)/2 mod 2^64, exactly.
uint64_t tri64(uint64_t m) { return (m & 1) ? m * ((m - 1) >> 1) : (m >> 1) * (m - 1); }

// Phase of tone t at absolute sample m: phi0 + m inc (+ K m(m-1)/2 if chirped).
uint64_t ddc_phase_at(const rf_ddc *p, int t, uint64_t m)
{
    uint64_t ph = p->h_phi0[t] + m * p->h_inc[t];
    if (p->h_chirp) ph += p->h_chirp[t] * tri64(m);
    return ph;
}

struct DdcPlan {
    uint64_t nskip, neff, nout, keep_from, keep_len, skip_after;
};

DdcPlan ddc_plan(const rf_ddc *p, uint64_t n)
{
    DdcPlan r{};
    r.nskip = p->skip < n ? p->skip : n;
    r.neff = n - r.nskip;
    const uint64_t vlen = (uint64_t)p->H + r.neff;
    if (p->skip > n) {
        r.skip_after = p->skip - n;
        return r;
    }
    r.nout = vlen >= (uint64_t)p->T ? (vlen - p->T) / p->D + 1 : 0;
    const uint64_t consumed = r.nout * (uint64_t)p->D;
    if (consumed <= vlen) {
        r.keep_from = consumed;
        r.keep_len = vlen - consumed;
    } else {
        r.skip_after = consumed - vlen;
    }
    return r;
}

}  // namespace

namespace rfi {

int ddc_prepare(rf_ddc *p, const int16_t *iq_dev, uint64_t nsamples, float *out_dev, uint64_t ld,
                rfk::DdcLaunch *a, uint64_t *nout)
{
    if (!p) return fail(RF_EINVAL, "ddc_process: handle is NULL");
    if (nsamples > p->max_samples)
        return fail(RF_EINVAL, "ddc_process: nsamples=%llu exceeds max_samples_per_call=%llu",
                    (unsigned long long)nsamples, (unsigned long long)p->max_samples);
    if (nsamples > 0 && (!iq_dev || !aligned(iq_dev, 4)))
        return fail(RF_EINVAL, "ddc_process: iq_dev must be a non-NULL 4-byte aligned device pointer");
    const DdcPlan pl = ddc_plan(p, nsamples);
    if (pl.nout > 0) {
        if (ld < pl.nout)
            return fail(RF_ECAPACITY, "ddc_process: ld=%llu < %llu outputs", (unsigned long long)ld,
                        (unsigned long long)pl.nout);
        if (!out_dev || !aligned(out_dev, 8))
            return fail(RF_EINVAL, "ddc_process: out_dev must be a non-NULL 8-byte aligned device pointer");
    }
    a->vs.hist = p->d_hist[p->cur];
    a->vs.in = reinterpret_cast<const uint32_t *>(iq_dev) + pl.nskip;
    a->vs.H = p->skip > 0 ? 0 : p->H;
    a->vs.n = (int64_t)pl.neff;
    a->hist_out = p->d_hist[p->cur ^ 1];
    a->keep_from = (int64_t)pl.keep_from;
    a->keep_len = (int64_t)pl.keep_len;
    a->out = out_dev;
    a->ld = (int64_t)ld;
    a->wrev = p->d_wrev;
    a->inc = p->d_inc;
    a->phi0 = p->d_phi0;
    a->chirp = p->d_chirp;
    a->sintab = p->d_tab;
    a->base_abs = p->nnext * (uint64_t)p->D;
    a->nout = (int64_t)pl.nout;
    a->phase_out = p->d_phase;
    a->phase_at = p->S + nsamples;
    a->T = p->T;
    a->D = p->D;
    a->ntones = p->ntones;
    const int wg = p->ntones <= 64 ? 64 : p->ntones <= 128 ? 128 : p->ntones <= 256 ? 256
                   : p->ntones <= 512 ? 512 : 1024;
    const int64_t items = (int64_t)((p->ntones + wg - 1) / wg) * (int64_t)pl.nout;
    int64_t grid = p->grid > 0 ? p->grid : p->cus;
    if (grid > items) grid = items;
    if (grid < 1) grid = 1;
    a->grid = (int32_t)grid;
    *nout = pl.nout;
    return RF_OK;
}

void ddc_commit(rf_ddc *p, uint64_t nsamples, hipStream_t s)
{
    const DdcPlan pl = ddc_plan(p, nsamples);
    p->order.after(s);
    p->cur ^= 1;
    p->S += nsamples;
    p->nnext += pl.nout;
    p->H = (int64_t)pl.keep_len;
    p->skip = pl.skip_after;
}

int ddc_device(const rf_ddc *p) { return p->device; }
int ddc_ntones(const rf_ddc *p) { return p->ntones; }
size_t ddc_footprint(int ntones, int T)
{
    return (size_t)ntones * 8 * 3 + (size_t)T * 4 + (size_t)rfk::kSinTabLen * 4 + 2 * (size_t)T * 4;
}

}  // namespace rfi

namespace {

// Quarter-wave (cos, sin) pair table: entry r in [0, 2^14) holds
// (q[2^14 - r], q[r]) with q[j] = fp32(sin(pi j / 2^15)), i.e. the FP32
// (cos, sin) of 2 pi r / 2^16; the other three quadrants follow from it by
// exact sign changes and swaps.
void fill_sintab(float *tab)
{
    const double pi = 3.14159265358979323846264338327950288;
    for (int r = 0; r < rfk::kSinTabLen / 2; ++r) {
        tab[2 * r] = (float)sin(pi * (double)((1 << 14) - r) / 32768.0);
        tab[2 * r + 1] = (float)sin(pi * (double)r / 32768.0);
    }
}

}  // namespace

extern "C" {

int ddc_create(rf_ddc_t *out, int32_t ntones, const uint64_t *phase_inc, const uint64_t *phase0, int32_t ntaps,
               const float *lpf, int32_t decim, uint64_t max_samples_per_call)
{
    return ddc_create_chirp(out, ntones, phase_inc, phase0, nullptr, ntaps, lpf, decim, max_samples_per_call);
}

int ddc_create_chirp(rf_ddc_t *out, int32_t ntones, const uint64_t *phase_inc, const uint64_t *phase0,
                     const uint64_t *chirp, int32_t ntaps, const float *lpf, int32_t decim,
                     uint64_t max_samples_per_call)
{
    if (!out) return fail(RF_EINVAL, "ddc_create: out is NULL");
    *out = nullptr;
    if (ntones < 1 || ntones > 65536) return fail(RF_EINVAL, "ddc_create: ntones=%d must be in [1, 65536]", ntones);
    if (!phase_inc) return fail(RF_EINVAL, "ddc_create: phase_inc is NULL");
    if (ntaps < 1 || ntaps > 4096) return fail(RF_EINVAL, "ddc_create: ntaps=%d must be in [1, 4096]", ntaps);
    if (!lpf) return fail(RF_EINVAL, "ddc_create: lpf is NULL");
    if (decim < 1 || decim > (1 << 20)) return fail(RF_EINVAL, "ddc_create: decim=%d must be in [1, 2^20]", decim);
    if (max_samples_per_call < 1 || max_samples_per_call > (1ull << 40))
        return fail(RF_EINVAL, "ddc_create: max_samples_per_call out of range");
    for (int i = 0; i < ntaps; ++i)
        if (!isfinite(lpf[i])) return fail(RF_EINVAL, "ddc_create: lpf[%d] is not finite", i);

    rf_ddc *p = new (std::nothrow) rf_ddc;
    if (!p) return fail(RF_ENOMEM, "ddc_create: host allocation");
    p->ntones = ntones;
    p->T = ntaps;
    p->D = decim;
    p->max_samples = max_samples_per_call;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        ddc_free(p);
        return hip_fail(e, "hipGetDevice");
    }
    p->cus = device_cus(p->device);
    p->h_inc = (uint64_t *)malloc(sizeof(uint64_t) * ntones);
    p->h_phi0 = (uint64_t *)calloc(ntones, sizeof(uint64_t));
    p->h_taps = (float *)malloc(sizeof(float) * ntaps);
    float *wrev = (float *)malloc(sizeof(float) * ntaps);
    float *tab = (float *)malloc(sizeof(float) * rfk::kSinTabLen);
    if (chirp) p->h_chirp = (uint64_t *)malloc(sizeof(uint64_t) * ntones);
    if (!p->h_inc || !p->h_phi0 || !p->h_taps || !wrev || !tab || (chirp && !p->h_chirp)) {
        free(wrev);
        free(tab);
        ddc_free(p);
        return fail(RF_ENOMEM, "ddc_create: host allocation");
    }
    memcpy(p->h_inc, phase_inc, sizeof(uint64_t) * ntones);
    if (phase0) memcpy(p->h_phi0, phase0, sizeof(uint64_t) * ntones);
    if (chirp) memcpy(p->h_chirp, chirp, sizeof(uint64_t) * ntones);
    memcpy(p->h_taps, lpf, sizeof(float) * ntaps);
    for (int j = 0; j < ntaps; ++j) wrev[j] = lpf[ntaps - 1 - j];
    fill_sintab(tab);
    int rc = RF_OK;
    const size_t hist_len = (size_t)ntaps;
    if ((rc = dev_alloc(&p->d_inc, ntones, "inc")) || (rc = dev_alloc(&p->d_phi0, ntones, "phi0")) ||
        (rc = dev_alloc(&p->d_phase, ntones, "phase")) || (rc = dev_alloc(&p->d_wrev, ntaps, "taps")) ||
        (rc = dev_alloc(&p->d_tab, rfk::kSinTabLen, "table")) ||
        (rc = dev_alloc(&p->d_hist[0], hist_len, "history")) ||
        (rc = dev_alloc(&p->d_hist[1], hist_len, "history")) ||
        (chirp && (rc = dev_alloc(&p->d_chirp, ntones, "chirp")))) {
        free(wrev);
        free(tab);
        ddc_free(p);
        return rc;
    }
    e = hipMemcpy(p->d_inc, p->h_inc, sizeof(uint64_t) * ntones, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_phi0, p->h_phi0, sizeof(uint64_t) * ntones, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_phase, p->h_phi0, sizeof(uint64_t) * ntones, hipMemcpyHostToDevice);
    if (e == hipSuccess && chirp)
        e = hipMemcpy(p->d_chirp, p->h_chirp, sizeof(uint64_t) * ntones, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_wrev, wrev, sizeof(float) * ntaps, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_tab, tab, sizeof(float) * rfk::kSinTabLen, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->order.ev, hipEventDisableTiming);
    free(wrev);
    free(tab);
    if (e != hipSuccess) {
        ddc_free(p);
        return hip_fail(e, "ddc_create");
    }
    const char *g = getenv("RFCHAN_DDC_GRID");
    if (g) p->grid = atoi(g);
    *out = p;
    return RF_OK;
}

uint64_t ddc_outputs_for(rf_ddc_t p, uint64_t nsamples)
{
    if (!p) return 0;
    return ddc_plan(p, nsamples).nout;
}

int ddc_process(rf_ddc_t p, const int16_t *iq_dev, uint64_t nsamples, float *out_dev, uint64_t ld, uint64_t *nout,
                void *hip_stream)
{
    if (nout) *nout = 0;
    rfk::DdcLaunch a;
    uint64_t no = 0;
    int rc = rfi::ddc_prepare(p, iq_dev, nsamples, out_dev, ld, &a, &no);
    if (rc || nsamples == 0) return rc;

    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    rc = p->order.before(s);
    if (rc) return rc;
    HIP_TRY(rfk::launch_ddc(a, s), "ddc kernel launch");
    rfi::ddc_commit(p, nsamples, s);
    if (nout) *nout = no;
    return RF_OK;
}

int ddc_get_phase(rf_ddc_t p, uint64_t *phase_host)
{
    if (!p || !phase_host) return fail(RF_EINVAL, "ddc_get_phase: NULL argument");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    HIP_TRY(hipMemcpy(phase_host, p->d_phase, sizeof(uint64_t) * p->ntones, hipMemcpyDeviceToHost),
            "hipMemcpy(phase)");
    return RF_OK;
}

int ddc_counters(rf_ddc_t p, uint64_t *samples_in, uint64_t *outputs_out, uint64_t *history_samples)
{
    if (!p) return fail(RF_EINVAL, "ddc_counters: handle is NULL");
    if (samples_in) *samples_in = p->S;
    if (outputs_out) *outputs_out = p->nnext;
    if (history_samples) *history_samples = (uint64_t)p->H;
    return RF_OK;
}

int ddc_get_state(rf_ddc_t p, void *blob, size_t *size)
{
    if (!p || !size) return fail(RF_EINVAL, "ddc_get_state: NULL argument");
    const size_t need = sizeof(DdcStateBlob) + (size_t)p->H * 4;
    if (!blob) {
        *size = need;
        return RF_OK;
    }
    if (*size < need) {
        *size = need;
        return fail(RF_ECAPACITY, "ddc_get_state: blob needs %zu bytes", need);
    }
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    DdcStateBlob h = {kDdcMagic, 1, p->ntones, p->T, p->D, 0, p->S, p->nnext, p->skip, p->H, ddc_fingerprint(p)};
    memcpy(blob, &h, sizeof h);
    if (p->H > 0)
        HIP_TRY(hipMemcpy((char *)blob + sizeof h, p->d_hist[p->cur], (size_t)p->H * 4, hipMemcpyDeviceToHost),
                "hipMemcpy(state)");
    *size = need;
    return RF_OK;
}

int ddc_set_state(rf_ddc_t p, const void *blob, size_t size)
{
    if (!p || !blob) return fail(RF_EINVAL, "ddc_set_state: NULL argument");
    DdcStateBlob h;
    if (size < sizeof h) return fail(RF_EINVAL, "ddc_set_state: blob too small");
    memcpy(&h, blob, sizeof h);
    if (h.magic != kDdcMagic || h.version != 1) return fail(RF_EINVAL, "ddc_set_state: not a DDC state blob");
    if (h.fingerprint != ddc_fingerprint(p)) return fail(RF_EINVAL, "ddc_set_state: blob is for another bank");
    if (h.H < 0 || h.H >= p->T || size < sizeof h + (size_t)h.H * 4)
        return fail(RF_EINVAL, "ddc_set_state: inconsistent history length");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    if (h.H > 0)
        HIP_TRY(hipMemcpy(p->d_hist[p->cur], (const char *)blob + sizeof h, (size_t)h.H * 4, hipMemcpyHostToDevice),
                "hipMemcpy(state)");
    // phase of the next sample follows from the sample count
    uint64_t *ph = (uint64_t *)malloc(sizeof(uint64_t) * p->ntones);
    if (!ph) return fail(RF_ENOMEM, "ddc_set_state: host allocation");
    for (int t = 0; t < p->ntones; ++t) ph[t] = ddc_phase_at(p, t, h.S);
    hipError_t e = hipMemcpy(p->d_phase, ph, sizeof(uint64_t) * p->ntones, hipMemcpyHostToDevice);
    free(ph);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(phase)");
    p->S = h.S;
    p->nnext = h.nnext;
    p->skip = h.skip;
    p->H = h.H;
    return RF_OK;
}

int ddc_reset(rf_ddc_t p)
{
    if (!p) return fail(RF_EINVAL, "ddc_reset: handle is NULL");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    HIP_TRY(hipMemcpy(p->d_phase, p->h_phi0, sizeof(uint64_t) * p->ntones, hipMemcpyHostToDevice),
            "hipMemcpy(phase)");
    p->S = 0;
    p->nnext = 0;
    p->H = 0;
    p->skip = 0;
    return RF_OK;
}

int ddc_destroy(rf_ddc_t p)
{
    if (!p) return RF_OK;
    int rc = RF_OK;
    {
        DeviceGuard dg(p->device);
        if (dg.err == hipSuccess) rc = p->order.sync();
        ddc_free(p);
    }
    return rc;
}

}  // extern "C"

// ================================================================ autotuner
//
// Candidate launch configurations are timed with HIP events on scratch
// buffers (the handle's history, phase and counters are not touched); the
// fastest is kept in the handle and appended to a plain-text cache
// (RFCHAN_TUNE_CACHE, default $HOME/.cache/rfchan_tune.txt), one line per
// "kind arch key... choice... microseconds", which *_create consults.

namespace {

// Bytes of scratch the tuner spreads its launches over (eight times the
// MI355X's 256 MB last-level cache, so that a launch's data is no longer
// cached when it comes round again and timings reflect HBM streaming), capped
// at a quarter of the free device memory.
constexpr uint64_t kTuneFootprint = 2048ull << 20;

uint64_t tune_footprint()
{
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return 512ull << 20;
    const uint64_t q = (uint64_t)fr / 4;
    return q < kTuneFootprint ? q : kTuneFootprint;
}

std::string tune_cache_path()
{
    const char *p = getenv("RFCHAN_TUNE_CACHE");
    if (p && *p) return p;
    const char *h = getenv("HOME");
    return std::string(h ? h : ".") + "/.cache/rfchan_tune.txt";
}

std::string device_arch(int dev)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Last cache line matching the key; returns the numbers after the key.
bool tune_lookup(const std::string &key, long *v, int nv)
{
    FILE *f = fopen(tune_cache_path().c_str(), "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        if (strncmp(line, key.c_str(), key.size()) != 0 || line[key.size()] != ' ') continue;
        const char *q = line + key.size();
        long tmp[8];
        int got = 0;
        for (; got < nv && got < 8; ++got) {
            char *end = nullptr;
            tmp[got] = strtol(q, &end, 10);
            if (end == q) break;
            q = end;
        }
        if (got == nv) {
            for (int i = 0; i < nv; ++i) v[i] = tmp[i];
            found = true;
        }
    }
    fclose(f);
    return found;
}

void tune_store(const std::string &key, const long *v, int nv, double us)
{
    std::string path = tune_cache_path();
    size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);  // best effort
    FILE *f = fopen(path.c_str(), "a");
    if (!f) return;
    fprintf(f, "%s", key.c_str());
    for (int i = 0; i < nv; ++i) fprintf(f, " %ld", v[i]);
    fprintf(f, " %.3f\n", us);
    fclose(f);
}

std::string pfb_key(const rf_pfb *p, uint64_t n)
{
    char b[128];
    snprintf(b, sizeof b, "pfb %s %d %d %d %llu", device_arch(p->device).c_str(), p->N, p->M, p->mode,
             (unsigned long long)n);
    return b;
}

std::string ddc_key(const rf_ddc *p, uint64_t n)
{
    char b[128];
    snprintf(b, sizeof b, "ddc %s %d %d %d %llu", device_arch(p->device).c_str(), p->ntones, p->T, p->D,
             (unsigned long long)n);
    return b;
}

// Average duration (us) of `reps` launches of `fn` on stream s.
template <typename Fn>
int time_launches(hipStream_t s, int reps, Fn fn, double *us)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0), "hipEventCreate");
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    e = fn();   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = fn();
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "tuning launch");
    *us = ms * 1e3 / reps;
    return RF_OK;
}

}  // namespace

extern "C" {

int pfb_tune(rf_pfb_t p, uint64_t nsamples, void *hip_stream, double *best_us)
{
    if (!p || nsamples < (uint64_t)p->N * p->M || nsamples > p->max_samples)
        return fail(RF_EINVAL, "pfb_tune: need a handle and N*M <= nsamples <= max_samples_per_call");
    if (p->large) return fail(RF_EUNSUPPORTED, "pfb_tune: large-N banks have no tunable launch shape");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = p->order.sync();
    if (rc) return rc;
    const uint64_t F = (nsamples - (uint64_t)p->N * p->M) / p->N + 1;
    // Rotate over enough scratch copies that their traffic exceeds the 256 MB
    // last-level cache several times over, as a long stream does.
    const uint64_t per = nsamples * 4 + F * p->N * 8;
    int copies = (int)((tune_footprint() + per - 1) / per);
    if (copies < 1) copies = 1;
    if (copies > 64) copies = 64;
    uint32_t *in = nullptr, *hist = nullptr;
    float *out = nullptr;
    if ((rc = dev_alloc(&in, nsamples * copies, "tune input")) ||
        (rc = dev_alloc(&hist, (size_t)p->N * p->M, "tune history")) ||
        (rc = dev_alloc(&out, 2 * F * p->N * copies, "tune output"))) {
        (void)hipFree(in);
        (void)hipFree(hist);
        return rc;
    }
    (void)rfk::fill_iq(in, nsamples * copies, s);
    rfk::PfbLaunch a{};
    a.vs.hist = hist;
    a.vs.H = 0;
    a.vs.n = (int64_t)nsamples;
    a.hist_out = hist;
    a.keep_from = (int64_t)F * p->N;
    a.keep_len = (int64_t)nsamples - a.keep_from;
    a.taps = p->d_taps;
    a.tw = p->d_tw;
    a.F = (int64_t)F;
    a.N = p->N;
    a.M = p->M;
    static const int rls[] = {8, 12, 16, 20, 24, 28, 32, 48, 64};
    // kernel variants tried: for N = 1024, M = 8 single or double-buffered
    // LDS, each with forward runs or with alternate runs walked backwards;
    // for N = 256, 512, 2048 at M = 4, 8 and N = 1024 at M = 4 the two run orders
    static const int vars8[] = {0, 1, 16, 17}, vars2[] = {0, 16};
    const bool fft = p->mode == RF_DFT_FFT_F32;
    const bool v4 = fft && p->N == 1024 && p->M == 8;
    const bool v2 = fft && !v4 && (p->M == 4 || p->M == 8) &&
                    (p->N == 256 || p->N == 512 || p->N == 1024 || p->N == 2048);
    const int *vars = v4 ? vars8 : vars2;
    const int nvar = v4 ? 4 : v2 ? 2 : 1;
    double best = 1e30;
    int best_rl = 0, best_var = 0;
    int k = 0;
    // two passes over every shape (best of both), so a clock ramp or a
    // transient does not decide the choice
    for (int pass = 0; pass < 2 && rc == RF_OK; ++pass)
    for (int rl : rls) {
        for (int vi = 0; vi < nvar; ++vi) {
            const int var = vars[vi];
            a.run_len = rl;
            a.variant = var;
            double us = 0;
            rc = time_launches(s, 2 * copies, [&]() {
                a.vs.in = in + (size_t)(k % copies) * nsamples;
                a.out = out + (size_t)(k % copies) * 2 * F * p->N;
                ++k;
                return p->mode == RF_DFT_FFT_F32
                           ? rfk::launch_pfb(a, s)
                           : rfk::launch_pfb_mfma(a, p->mode == RF_DFT_MFMA_BF16X2 ? rfk::RF_PREC_BF16 : rfk::RF_PREC_F16, s);
            }, &us);
            if (rc) break;
            if (us < best) {
                best = us;
                best_rl = rl;
                best_var = var;
            }
        }
        if (rc) break;
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(in);
    (void)hipFree(hist);
    (void)hipFree(out);
    if (rc) return rc;
    p->run_len = best_rl;
    p->variant = best_var;
    const long v[2] = {best_rl, best_var};
    tune_store(pfb_key(p, nsamples), v, 2, best);
    if (best_us) *best_us = best;
    return RF_OK;
}

int pfb_tuned_config(rf_pfb_t p, int32_t *run_len, int32_t *variant)
{
    if (!p) return fail(RF_EINVAL, "pfb_tuned_config: handle is NULL");
    if (run_len) *run_len = p->run_len;
    if (variant) *variant = p->variant;
    return RF_OK;
}

int ddc_tune(rf_ddc_t p, uint64_t nsamples, void *hip_stream, double *best_us)
{
    if (!p || nsamples < (uint64_t)p->T || nsamples > p->max_samples)
        return fail(RF_EINVAL, "ddc_tune: need a handle and T <= nsamples <= max_samples_per_call");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = p->order.sync();
    if (rc) return rc;
    const uint64_t nout = (nsamples - p->T) / p->D + 1;
    uint32_t *in = nullptr, *hist = nullptr;
    float *out = nullptr;
    uint64_t *phase = nullptr;
    if ((rc = dev_alloc(&in, nsamples, "tune input")) || (rc = dev_alloc(&hist, (size_t)p->T, "tune history")) ||
        (rc = dev_alloc(&out, 2 * nout * p->ntones, "tune output")) ||
        (rc = dev_alloc(&phase, p->ntones, "tune phase"))) {
        (void)hipFree(in);
        (void)hipFree(hist);
        (void)hipFree(out);
        return rc;
    }
    (void)rfk::fill_iq(in, nsamples, s);
    rfk::DdcLaunch a{};
    a.vs.hist = hist;
    a.vs.in = in;
    a.vs.H = 0;
    a.vs.n = (int64_t)nsamples;
    a.hist_out = hist;
    a.keep_from = (int64_t)(nout * p->D);
    a.keep_len = (int64_t)nsamples - a.keep_from;
    if (a.keep_len < 0) a.keep_len = 0;
    a.out = out;
    a.ld = (int64_t)nout;
    a.wrev = p->d_wrev;
    a.inc = p->d_inc;
    a.phi0 = p->d_phi0;
    a.chirp = p->d_chirp;
    a.sintab = p->d_tab;
    a.base_abs = 0;
    a.nout = (int64_t)nout;
    a.phase_out = phase;
    a.phase_at = nsamples;
    a.T = p->T;
    a.D = p->D;
    a.ntones = p->ntones;
    const int grids[] = {p->cus / 2, p->cus, 2 * p->cus, 4 * p->cus};
    double best = 1e30;
    int best_grid = p->cus;
    for (int g : grids) {
        if (g < 1) continue;
        a.grid = g;
        double us = 0;
        rc = time_launches(s, 3, [&]() { return rfk::launch_ddc(a, s); }, &us);
        if (rc) break;
        if (us < best) {
            best = us;
            best_grid = g;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(in);
    (void)hipFree(hist);
    (void)hipFree(out);
    (void)hipFree(phase);
    if (rc) return rc;
    p->grid = best_grid;
    const long v[1] = {best_grid};
    tune_store(ddc_key(p, nsamples), v, 1, best);
    if (best_us) *best_us = best;
    return RF_OK;
}

int ddc_tuned_config(rf_ddc_t p, int32_t *grid)
{
    if (!p) return fail(RF_EINVAL, "ddc_tuned_config: handle is NULL");
    if (grid) *grid = p->grid;
    return RF_OK;
}

int pfb_apply_tuned(rf_pfb_t p, uint64_t nsamples)
{
    if (!p) return fail(RF_EINVAL, "pfb_apply_tuned: handle is NULL");
    long v[2];
    if (!tune_lookup(pfb_key(p, nsamples), v, 2)) return RF_EAGAIN;
    if (v[0] < 4 || v[0] % 4) return fail(RF_EINVAL, "pfb_apply_tuned: corrupt cache entry");
    p->run_len = (int)v[0];
    p->variant = (int)v[1];
    return RF_OK;
}

int ddc_apply_tuned(rf_ddc_t p, uint64_t nsamples)
{
    if (!p) return fail(RF_EINVAL, "ddc_apply_tuned: handle is NULL");
    long v[1];
    if (!tune_lookup(ddc_key(p, nsamples), v, 1)) return RF_EAGAIN;
    if (v[0] < 1) return fail(RF_EINVAL, "ddc_apply_tuned: corrupt cache entry");
    p->grid = (int)v[0];
    return RF_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ Tx

struct rf_tx {
    int ntones = 0;
    uint64_t max_samples = 0;
    int device = 0;
    // device oscillator state (ping-pong: a call reads cur and writes cur^1)
    uint64_t *d_phase[2] = {nullptr, nullptr}, *d_rate[2] = {nullptr, nullptr};
    uint64_t *d_chirp = nullptr;
    float *d_amp = nullptr, *d_tab = nullptr;
    int cur = 0;
    bool chirped = false;
    uint64_t S = 0;   // samples produced
    // creation state, for tx_reset
    uint64_t *h_phase0 = nullptr, *h_rate0 = nullptr, *h_chirp0 = nullptr;
    float *h_amp0 = nullptr;
    StreamOrder order;
};

namespace {

void tx_free(rf_tx *p)
{
    if (!p) return;
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(p->d_phase[i]);
        (void)hipFree(p->d_rate[i]);
    }
    (void)hipFree(p->d_chirp);
    (void)hipFree(p->d_amp);
    (void)hipFree(p->d_tab);
    if (p->order.ev) (void)hipEventDestroy(p->order.ev);
    free(p->h_phase0);
    free(p->h_rate0);
    free(p->h_chirp0);
    free(p->h_amp0);
    delete p;
}

// Half-wave sine table S[i] = sin(2 pi i / 2^16), i < 2^15, from the quarter
// wave q[j] = fp32(sin(pi j / 2^15)) by symmetry.
void fill_halfwave(float *tab)
{
    const double pi = 3.14159265358979323846264338327950288;
    for (int i = 0; i < rfk::kSinTabLen; ++i) {
        const int j = i <= (1 << 14) ? i : (1 << 15) - i;
        tab[i] = (float)sin(pi * (double)j / 32768.0);
    }
}

int tx_upload_state(rf_tx *p)
{
    const size_t b = sizeof(uint64_t) * p->ntones;
    HIP_TRY(hipMemcpy(p->d_phase[p->cur], p->h_phase0, b, hipMemcpyHostToDevice), "hipMemcpy(phase)");
    HIP_TRY(hipMemcpy(p->d_rate[p->cur], p->h_rate0, b, hipMemcpyHostToDevice), "hipMemcpy(rate)");
    if (p->d_chirp) HIP_TRY(hipMemcpy(p->d_chirp, p->h_chirp0, b, hipMemcpyHostToDevice), "hipMemcpy(chirp)");
    HIP_TRY(hipMemcpy(p->d_amp, p->h_amp0, sizeof(float) * p->ntones, hipMemcpyHostToDevice), "hipMemcpy(amp)");
    return RF_OK;
}

}  // namespace

extern "C" {

int tx_create(rf_tx_t *out, int32_t ntones, const uint64_t *phase_inc, const uint64_t *phase0,
              const uint64_t *chirp, const float *amplitude, uint64_t max_samples_per_call)
{
    if (!out) return fail(RF_EINVAL, "tx_create: out is NULL");
    *out = nullptr;
    if (ntones < 1 || ntones > 65536) return fail(RF_EINVAL, "tx_create: ntones=%d must be in [1, 65536]", ntones);
    if (!phase_inc || !amplitude) return fail(RF_EINVAL, "tx_create: phase_inc and amplitude are required");
    if (max_samples_per_call < 1 || max_samples_per_call > (1ull << 40))
        return fail(RF_EINVAL, "tx_create: max_samples_per_call out of range");
    for (int i = 0; i < ntones; ++i)
        if (!isfinite(amplitude[i])) return fail(RF_EINVAL, "tx_create: amplitude[%d] is not finite", i);
    rf_tx *p = new (std::nothrow) rf_tx;
    if (!p) return fail(RF_ENOMEM, "tx_create: host allocation");
    p->ntones = ntones;
    p->max_samples = max_samples_per_call;
    p->chirped = chirp != nullptr;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        tx_free(p);
        return hip_fail(e, "hipGetDevice");
    }
    const size_t b = sizeof(uint64_t) * ntones;
    p->h_phase0 = (uint64_t *)calloc(ntones, sizeof(uint64_t));
    p->h_rate0 = (uint64_t *)malloc(b);
    p->h_chirp0 = (uint64_t *)calloc(ntones, sizeof(uint64_t));
    p->h_amp0 = (float *)malloc(sizeof(float) * ntones);
    float *tab = (float *)malloc(sizeof(float) * rfk::kSinTabLen);
    if (!p->h_phase0 || !p->h_rate0 || !p->h_chirp0 || !p->h_amp0 || !tab) {
        free(tab);
        tx_free(p);
        return fail(RF_ENOMEM, "tx_create: host allocation");
    }
    if (phase0) memcpy(p->h_phase0, phase0, b);
    memcpy(p->h_rate0, phase_inc, b);
    if (chirp) memcpy(p->h_chirp0, chirp, b);
    memcpy(p->h_amp0, amplitude, sizeof(float) * ntones);
    fill_halfwave(tab);
    int rc = RF_OK;
    if ((rc = dev_alloc(&p->d_phase[0], ntones, "tx phase")) || (rc = dev_alloc(&p->d_phase[1], ntones, "tx phase")) ||
        (rc = dev_alloc(&p->d_rate[0], ntones, "tx rate")) || (rc = dev_alloc(&p->d_rate[1], ntones, "tx rate")) ||
        (rc = dev_alloc(&p->d_amp, ntones, "tx amplitude")) || (rc = dev_alloc(&p->d_tab, rfk::kSinTabLen, "tx table")) ||
        (chirp && (rc = dev_alloc(&p->d_chirp, ntones, "tx chirp")))) {
        free(tab);
        tx_free(p);
        return rc;
    }
    e = hipMemcpy(p->d_tab, tab, sizeof(float) * rfk::kSinTabLen, hipMemcpyHostToDevice);
    free(tab);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->order.ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        tx_free(p);
        return hip_fail(e, "tx_create");
    }
    if ((rc = tx_upload_state(p))) {
        tx_free(p);
        return rc;
    }
    *out = p;
    return RF_OK;
}

int tx_synthesize(rf_tx_t p, int16_t *out_dev, uint64_t nsamples, void *hip_stream)
{
    if (!p) return fail(RF_EINVAL, "tx_synthesize: handle is NULL");
    if (nsamples > p->max_samples)
        return fail(RF_EINVAL, "tx_synthesize: nsamples=%llu exceeds max_samples_per_call=%llu",
                    (unsigned long long)nsamples, (unsigned long long)p->max_samples);
    if (nsamples == 0) return RF_OK;
    if (!out_dev) return fail(RF_EINVAL, "tx_synthesize: out_dev is NULL");
    if ((uintptr_t)out_dev & 3) return fail(RF_EINVAL, "tx_synthesize: out_dev must be 4-byte aligned");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = p->order.before(s);
    if (rc) return rc;
    rfk::TxLaunch a{};
    a.out = (uint32_t *)out_dev;
    a.n = (int64_t)nsamples;
    a.phase = p->d_phase[p->cur];
    a.rate = p->d_rate[p->cur];
    a.chirp = p->d_chirp;
    a.amp = p->d_amp;
    a.halftab = p->d_tab;
    a.phase_out = p->d_phase[p->cur ^ 1];
    a.rate_out = p->d_rate[p->cur ^ 1];
    a.ntones = p->ntones;
    HIP_TRY(rfk::launch_tx(a, s), "tx kernel launch");
    p->cur ^= 1;
    p->S += nsamples;
    p->order.after(s);
    return RF_OK;
}

int tx_set_tones(rf_tx_t p, const float *amplitude, const uint64_t *phase_inc, const uint64_t *chirp)
{
    if (!p) return fail(RF_EINVAL, "tx_set_tones: handle is NULL");
    if (chirp && !p->chirped) return fail(RF_EINVAL, "tx_set_tones: chirp words need a bank created with chirp");
    if (amplitude)
        for (int i = 0; i < p->ntones; ++i)
            if (!isfinite(amplitude[i])) return fail(RF_EINVAL, "tx_set_tones: amplitude[%d] is not finite", i);
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    const size_t b = sizeof(uint64_t) * p->ntones;
    if (amplitude)
        HIP_TRY(hipMemcpy(p->d_amp, amplitude, sizeof(float) * p->ntones, hipMemcpyHostToDevice), "hipMemcpy(amp)");
    if (phase_inc) HIP_TRY(hipMemcpy(p->d_rate[p->cur], phase_inc, b, hipMemcpyHostToDevice), "hipMemcpy(rate)");
    if (chirp) HIP_TRY(hipMemcpy(p->d_chirp, chirp, b, hipMemcpyHostToDevice), "hipMemcpy(chirp)");
    return RF_OK;
}

int tx_get_state(rf_tx_t p, uint64_t *phase, uint64_t *rate, uint64_t *samples)
{
    if (!p) return fail(RF_EINVAL, "tx_get_state: handle is NULL");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    const size_t b = sizeof(uint64_t) * p->ntones;
    if (phase) HIP_TRY(hipMemcpy(phase, p->d_phase[p->cur], b, hipMemcpyDeviceToHost), "hipMemcpy(phase)");
    if (rate) HIP_TRY(hipMemcpy(rate, p->d_rate[p->cur], b, hipMemcpyDeviceToHost), "hipMemcpy(rate)");
    if (samples) *samples = p->S;
    return RF_OK;
}

int tx_reset(rf_tx_t p)
{
    if (!p) return fail(RF_EINVAL, "tx_reset: handle is NULL");
    DeviceGuard dg(p->device);
    HIP_TRY(dg.err, "hipSetDevice");
    int rc = p->order.sync();
    if (rc) return rc;
    if ((rc = tx_upload_state(p))) return rc;
    p->S = 0;
    return RF_OK;
}

int tx_destroy(rf_tx_t p)
{
    if (!p) return RF_OK;
    int rc = RF_OK;
    {
        DeviceGuard dg(p->device);
        if (dg.err == hipSuccess) rc = p->order.sync();
        tx_free(p);
    }
    return rc;
}

}  // extern "C"
