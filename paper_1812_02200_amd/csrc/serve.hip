// serve.hip -- multi-stream serving core: admission by device-memory
// footprint, continuous batching, grouped persistent kernels, hipGraph replay.
//
// The paper's readout moves buffers between host threads through lock-free
// queues of pointers to pre-allocated memory and hands them to a GPU
// processing thread (Sec. III, Fig. 2).  Here one scheduler thread owns the
// GPU: clients queue buffers per stream, and the scheduler repeatedly takes
// the oldest queued buffer of every stream that has a free output slot, turns
// them into item tables (one per (N, M) class of PFB streams, one for all DDC
// banks), uploads the tables and launches one grouped kernel per table.  A
// stream's consecutive buffers land in consecutive batches on the same HIP
// stream, so its history and phase carry over without any host wait.  Up to
// two batches are in flight: while one runs, the next is prepared.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/rfchan.h"
#include "rf_handles.hpp"
#include "rf_internal.hpp"

namespace {

using rfi::set_error;

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    const int16_t *iq;
    uint64_t n;
    uint64_t tag;
    double t_submit;
    bool host = false;         // pinned host memory: staged before use
    int stage = -1;            // staging slot holding its copy (host requests, once issued)
};

struct Done {
    int stream, slot, stage;
    int tp = -1, td = -1;      // item tables (PFB, DDC) of a grouped batch, or -1
    bool reported = false;
    bool partial = false;      // a chunk of a long DDC call that is not its last: nothing to report
    Request req;
    uint64_t pfb_frames, ddc_outputs, ddc_ld;
    const float *pfb_out, *ddc_out;
    double t_launch;
};

struct Stream {
    int id = -1;
    int kinds = 0;
    rf_pfb *pfb = nullptr;
    rf_ddc *ddc = nullptr;
    int N = 0, M = 0, ntones = 0;
    uint64_t max_buffer = 0;
    uint64_t pfb_cap = 0;      // frames per output slot
    uint64_t ddc_ld = 0;       // outputs per tone per output slot
    int nslots = 0;
    std::vector<float *> pfb_slot, ddc_slot;
    std::vector<int> free_slots;
    // staging slots for pinned-host buffers: device copies, each with the
    // event that marks its copy's completion on the server's copy stream
    std::vector<uint32_t *> stage_buf;
    std::vector<hipEvent_t> stage_ev;
    std::vector<int> free_stage;
    // a long DDC call in progress, issued over several batches (grouped modes)
    struct Chunked {
        bool on = false;
        Done d{};
        rfk::DdcLaunch a{};
        int64_t units = 0, issued = 0;
    } ch;
    std::deque<Request> queue;
    int inflight = 0;
    size_t footprint = 0;
    bool closing = false;
};


// What one batch entry launches: the request's PFB part, and which of its DDC
// units (all, or a chunk); `final` entries complete the request.
struct Part {
    bool first = true;                   // the request's first entry (reads its input)
    bool pfb = false;
    int64_t ddc_off = 0, ddc_cnt = -1;   // -1: all units
    bool final = true;
};

// Work per DDC chunk in tap-tones (about a millisecond at the measured rate):
// a call with more than two chunks of work is issued over several batches so
// that light buffers that arrive meanwhile are not queued behind all of it.
constexpr double kDdcChunkWork = 3.5e9;

int64_t ddc_chunk_units(const rfk::DdcLaunch &a)
{
    const double per_unit = (double)rfk::ddc_group_wg(a.ntones) * (double)a.T;
    const int64_t u = (int64_t)(kDdcChunkWork / per_unit);
    return u < 1 ? 1 : u;
}

// Device/pinned layout of one batch's item tables.
struct Blob {
    void *host = nullptr;      // pinned
    void *dev = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;   // completion of the batch that last used this blob
    bool busy = false;
    double t_launch = 0;
    std::vector<Done> done;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_version = -1;
    // completion of each table's grouped kernel (recorded on its branch), so
    // that a request completes when its own kernels finish, not the batch's
    std::vector<hipEvent_t> tev;
};

}  // namespace

struct rfs_server {
    int device = 0;
    int mode = RFS_MODE_BATCHED;
    int max_streams = 64;
    int cus = 256;
    uint64_t budget = 0, admitted = 0;
    hipStream_t hs = nullptr;
    hipStream_t cs = nullptr;          // host-to-device copies of pinned-host buffers
    std::vector<hipStream_t> branch;   // branch streams of the batched mode's grouped launches
    std::vector<hipEvent_t> fork_ev;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::map<int, Stream *> streams;
    int next_id = 0;
    std::deque<rfs_completion> completions;
    std::thread thr;
    std::atomic<bool> stop{false};
    Blob blobs[2];
    int next_blob = 0;
    // class tables: distinct (N, M) of open PFB streams -> table index t,
    // then distinct DDC work-group sizes -> table C + index
    std::vector<std::pair<int, int>> classes;
    std::vector<int> ddc_classes;
    int class_version = 0;
    size_t region = 0;                 // bytes per table region
    rfs_stats st{};
    std::string fatal;
};

namespace {

constexpr int kMaxBranches = 4;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t region_bytes(int max_items)
{
    const size_t item = std::max(sizeof(rfk::PfbItem), sizeof(rfk::DdcItem));
    return align_up(sizeof(rfk::GroupHeader), 256) + align_up(item * (size_t)max_items, 256);
}

// Tables: [PFB class 0] ... [PFB class C-1] [DDC class 0] ... [DDC class D-1];
// C and D fixed by class_version.
rfk::GroupHeader *hdr_at(void *base, size_t region, int t)
{
    return reinterpret_cast<rfk::GroupHeader *>((char *)base + region * t);
}
template <typename ItemT>
ItemT *items_at(void *base, size_t region, int t)
{
    return reinterpret_cast<ItemT *>((char *)base + region * t + align_up(sizeof(rfk::GroupHeader), 256));
}

uint64_t slot_frames(int N, int M, uint64_t max_buffer) { return ((uint64_t)N * M + max_buffer) / N + 1; }
uint64_t slot_outputs(int T, int D, uint64_t max_buffer) { return ((uint64_t)T + max_buffer) / D + 2; }

size_t footprint_of(const rfs_stream_desc *d)
{
    size_t f = 0;
    const int slots = d->out_slots > 0 ? d->out_slots : 1;
    if (d->kinds & RFS_PFB) {
        f += rfi::pfb_footprint(d->nchan, d->ntaps, RF_DFT_FFT_F32);
        f += (size_t)slots * slot_frames(d->nchan, d->ntaps, d->max_buffer) * d->nchan * 8;
    }
    if (d->kinds & RFS_DDC) {
        f += rfi::ddc_footprint(d->ntones, d->lpf_taps);
        f += (size_t)slots * d->ntones * slot_outputs(d->lpf_taps, d->decim, d->max_buffer) * 8;
    }
    if (d->host_slots > 0) f += (size_t)d->host_slots * d->max_buffer * 4;
    return f;
}

void free_stream(Stream *s)
{
    if (!s) return;
    if (s->pfb) pfb_destroy(s->pfb);
    if (s->ddc) ddc_destroy(s->ddc);
    for (float *p : s->pfb_slot) (void)hipFree(p);
    for (float *p : s->ddc_slot) (void)hipFree(p);
    for (uint32_t *p : s->stage_buf) (void)hipFree(p);
    for (hipEvent_t e : s->stage_ev) (void)hipEventDestroy(e);
    delete s;
}

int class_index(rfs_server *S, int N, int M)
{
    for (size_t i = 0; i < S->classes.size(); ++i)
        if (S->classes[i].first == N && S->classes[i].second == M) return (int)i;
    return -1;
}

int ddc_class_index(rfs_server *S, int ntones)
{
    const int wg = rfk::ddc_group_wg(ntones);
    for (size_t i = 0; i < S->ddc_classes.size(); ++i)
        if (S->ddc_classes[i] == wg) return (int)i;
    return -1;
}

// Recompute the class lists from the open streams (caller holds mu).  A DDC
// bank is served by a work-group of its own size (one lane per tone, up to
// 1024), as in a single-stream launch.
void rebuild_classes(rfs_server *S)
{
    std::vector<std::pair<int, int>> c;
    std::vector<int> dc;
    for (auto &kv : S->streams) {
        if (kv.second->kinds & RFS_PFB) {
            std::pair<int, int> k(kv.second->N, kv.second->M);
            if (std::find(c.begin(), c.end(), k) == c.end()) c.push_back(k);
        }
        if (kv.second->kinds & RFS_DDC) {
            const int wg = rfk::ddc_group_wg(kv.second->ntones);
            if (std::find(dc.begin(), dc.end(), wg) == dc.end()) dc.push_back(wg);
        }
    }
    std::sort(c.begin(), c.end());
    std::sort(dc.begin(), dc.end());
    if (c != S->classes || dc != S->ddc_classes) {
        S->classes = c;
        S->ddc_classes = dc;
        ++S->class_version;
    }
}

int pfb_grid(rfs_server *S, int N) { return N >= 2048 ? S->cus : 2 * S->cus; }

// Build the batch graph for the current class lists into blob b: a table
// upload node, then one grouped-kernel node per PFB class and per DDC class
// (each depending on the upload only, so they may run side by side), each
// followed by an event-record node for that table.  The graph is assembled
// node by node rather than captured from a stream: a capture in progress on
// the scheduler's thread would make device-wide synchronisation in client
// threads fail.
int build_graph(rfs_server *S, Blob &b)
{
    if (b.exec) {
        (void)hipGraphExecDestroy(b.exec);
        b.exec = nullptr;
    }
    if (b.graph) {
        (void)hipGraphDestroy(b.graph);
        b.graph = nullptr;
    }
    const int C = (int)S->classes.size();
    const int NT = C + (int)S->ddc_classes.size();
    hipGraph_t g = nullptr;
    hipError_t err = hipGraphCreate(&g, 0);
    hipGraphNode_t up = nullptr;
    if (err == hipSuccess)
        err = hipGraphAddMemcpyNode1D(&up, g, nullptr, 0, b.dev, b.host, S->region * NT, hipMemcpyHostToDevice);
    for (int t = 0; t < NT && err == hipSuccess; ++t) {
        const rfk::GroupHeader *h = hdr_at(b.dev, S->region, t);
        const void *fn;
        int grid, block;
        const void *items;
        if (t < C) {
            fn = rfk::pfb_group_kernel(S->classes[t].first, S->classes[t].second);
            grid = pfb_grid(S, S->classes[t].first);
            block = rfk::pfb_group_wg_size(S->classes[t].first);
            items = items_at<rfk::PfbItem>(b.dev, S->region, t);
        } else {
            fn = rfk::ddc_group_kernel(S->ddc_classes[t - C]);
            grid = S->cus;
            block = S->ddc_classes[t - C];
            items = items_at<rfk::DdcItem>(b.dev, S->region, t);
        }
        if (!fn) {
            err = hipErrorInvalidValue;
            break;
        }
        void *args[] = {(void *)&h, (void *)&items};
        hipKernelNodeParams kp{};
        kp.func = const_cast<void *>(fn);
        kp.gridDim = dim3((unsigned)grid);
        kp.blockDim = dim3((unsigned)block);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t kn = nullptr, en = nullptr;
        err = hipGraphAddKernelNode(&kn, g, &up, 1, &kp);
        if (err == hipSuccess) err = hipGraphAddEventRecordNode(&en, g, &kn, 1, b.tev[t]);
    }
    if (err == hipSuccess) err = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
    if (err != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        b.exec = nullptr;
        (void)hipGetLastError();
        return set_error(RF_EDEVICE, "building the batch graph failed");
    }
    b.graph = g;
    b.graph_version = S->class_version;
    return RF_OK;
}

// Issue the host-to-device copies of queued pinned-host buffers, in queue
// order, into free staging slots (caller holds mu).  The copies run on the
// copy stream, overlapped with the batch in flight.
int stage_copies(rfs_server *S)
{
    for (auto &kv : S->streams) {
        Stream *s = kv.second;
        for (Request &r : s->queue) {
            if (!r.host || r.stage >= 0) continue;
            if (s->free_stage.empty()) break;
            const int k = s->free_stage.back();
            if (hipMemcpyAsync(s->stage_buf[k], r.iq, r.n * 4, hipMemcpyHostToDevice, S->cs) != hipSuccess ||
                hipEventRecord(s->stage_ev[k], S->cs) != hipSuccess)
                return set_error(RF_EDEVICE, "staging copy failed");
            s->free_stage.pop_back();
            r.stage = k;
        }
    }
    return RF_OK;
}

// Pick one request per eligible stream and prepare its launches (caller holds
// mu).  SEQUENTIAL mode takes only the oldest request overall.  A pinned-host
// request is eligible once its staging copy has been issued.
bool form_batch(rfs_server *S, std::vector<Done> &out, std::vector<rfk::PfbLaunch> &pl,
                std::vector<rfk::DdcLaunch> &dl, std::vector<Stream *> &who, std::vector<Part> &parts)
{
    const bool grouped = S->mode != RFS_MODE_SEQUENTIAL;
    std::vector<Stream *> cand;
    for (auto &kv : S->streams) {
        Stream *s = kv.second;
        if (s->ch.on ||
            (!s->queue.empty() && !s->free_slots.empty() && (!s->queue.front().host || s->queue.front().stage >= 0)))
            cand.push_back(s);
    }
    if (cand.empty()) return false;
    auto t_of = [](Stream *s) { return s->ch.on ? s->ch.d.req.t_submit : s->queue.front().t_submit; };
    std::sort(cand.begin(), cand.end(), [&](Stream *a, Stream *b) { return t_of(a) < t_of(b); });
    if (S->mode == RFS_MODE_SEQUENTIAL) cand.resize(1);
    for (Stream *s : cand) {
        if (s->ch.on) {   // the next chunk of a long DDC call
            Part pt;
            pt.first = false;
            pt.ddc_off = s->ch.issued;
            pt.ddc_cnt = std::min(ddc_chunk_units(s->ch.a), s->ch.units - s->ch.issued);
            s->ch.issued += pt.ddc_cnt;
            pt.final = s->ch.issued == s->ch.units;
            Done d = s->ch.d;
            d.partial = !pt.final;
            if (pt.final) s->ch.on = false;
            out.push_back(d);
            pl.push_back(rfk::PfbLaunch{});
            dl.push_back(s->ch.a);
            who.push_back(s);
            parts.push_back(pt);
            continue;
        }
        Request r = s->queue.front();
        const int slot = s->free_slots.back();
        Done d{};
        d.stream = s->id;
        d.slot = slot;
        d.stage = r.host ? r.stage : -1;
        d.req = r;
        if (r.host) r.iq = reinterpret_cast<const int16_t *>(s->stage_buf[r.stage]);
        rfk::PfbLaunch a{};
        rfk::DdcLaunch b{};
        bool ok = true;
        if (s->pfb) {
            uint64_t F = 0;
            ok = rfi::pfb_prepare(s->pfb, r.iq, r.n, s->pfb_slot[slot], s->pfb_cap, &a, &F) == RF_OK;
            d.pfb_frames = F;
            d.pfb_out = s->pfb_slot[slot];
        }
        if (ok && s->ddc) {
            uint64_t no = 0;
            ok = rfi::ddc_prepare(s->ddc, r.iq, r.n, s->ddc_slot[slot], s->ddc_ld, &b, &no) == RF_OK;
            d.ddc_outputs = no;
            d.ddc_ld = s->ddc_ld;
            d.ddc_out = s->ddc_slot[slot];
        }
        if (!ok) {   // cannot happen for validated submissions; drop the request with an error
            if (d.stage >= 0) s->free_stage.push_back(d.stage);
            s->queue.pop_front();
            rfs_completion c{};
            c.stream = s->id;
            c.slot = -1;
            c.tag = r.tag;
            c.nsamples = r.n;
            c.status = RF_EINVAL;
            c.t_submit = r.t_submit;
            c.t_done = now_s();
            S->completions.push_back(c);
            continue;
        }
        s->queue.pop_front();
        s->free_slots.pop_back();
        s->inflight++;
        Part pt;
        pt.pfb = s->pfb != nullptr;
        if (grouped && s->ddc && r.n) {
            const int64_t units = rfk::ddc_group_units(b), cu = ddc_chunk_units(b);
            if (units > 2 * cu) {   // long call: its first chunk now, the rest in later batches
                s->ch.on = true;
                s->ch.d = d;
                s->ch.a = b;
                s->ch.units = units;
                s->ch.issued = cu;
                pt.ddc_off = 0;
                pt.ddc_cnt = cu;
                pt.final = false;
                d.partial = true;
            }
        }
        out.push_back(d);
        pl.push_back(a);
        dl.push_back(b);
        who.push_back(s);
        parts.push_back(pt);
    }
    return !out.empty();
}

// Enqueue a batch.  Returns RF_OK or an error (GPU failure).
int launch_batch(rfs_server *S, Blob &b, std::vector<Done> &dn, std::vector<rfk::PfbLaunch> &pl,
                 std::vector<rfk::DdcLaunch> &dl, std::vector<Stream *> &who, const std::vector<Part> &parts)
{
    // the batch reads staged copies: wait for those copies (only)
    for (size_t i = 0; i < who.size(); ++i)
        if (dn[i].stage >= 0 && parts[i].first &&
            hipStreamWaitEvent(S->hs, who[i]->stage_ev[dn[i].stage], 0) != hipSuccess)
            return set_error(RF_EDEVICE, "wait for staging copy failed");
    // A batch of one request (the common case at light load) gains nothing
    // from item tables, grouped kernels or a graph: it is launched as the
    // single-stream kernels, which compute the same results bit for bit.
    if (S->mode == RFS_MODE_SEQUENTIAL || (who.size() == 1 && parts[0].ddc_cnt < 0)) {
        for (size_t i = 0; i < who.size(); ++i) {
            Stream *s = who[i];
            if (s->pfb && dn[i].req.n) {
                hipError_t e = rfk::launch_pfb(pl[i], S->hs);
                if (e != hipSuccess) return set_error(RF_EDEVICE, "pfb launch failed");
                rfi::pfb_commit(s->pfb, pl[i], dn[i].req.n, dn[i].pfb_frames, S->hs);
            }
            if (s->ddc && dn[i].req.n) {
                hipError_t e = rfk::launch_ddc(dl[i], S->hs);
                if (e != hipSuccess) return set_error(RF_EDEVICE, "ddc launch failed");
                rfi::ddc_commit(s->ddc, dn[i].req.n, S->hs);
            }
        }
        return RF_OK;
    }
    const int C = (int)S->classes.size();
    const int NT = C + (int)S->ddc_classes.size();
    for (int t = 0; t < NT; ++t) {
        rfk::GroupHeader *h = hdr_at(b.host, S->region, t);
        h->count = 0;
        h->total = 0;
    }
    for (size_t i = 0; i < who.size(); ++i) {
        Stream *s = who[i];
        if (!dn[i].req.n) continue;
        if (parts[i].pfb) {
            const int t = class_index(S, s->N, s->M);
            rfk::GroupHeader *h = hdr_at(b.host, S->region, t);
            rfk::PfbItem &it = items_at<rfk::PfbItem>(b.host, S->region, t)[h->count];
            it.a = pl[i];
            it.a.variant = 0;
            it.wg_begin = h->total;
            it.wgs = (int32_t)rfk::pfb_launch_wgs(pl[i]);
            h->total += it.wgs;
            h->count++;
            dn[i].tp = t;
        }
        if (s->ddc) {
            const int t = C + ddc_class_index(S, s->ntones);
            rfk::GroupHeader *h = hdr_at(b.host, S->region, t);
            rfk::DdcItem &it = items_at<rfk::DdcItem>(b.host, S->region, t)[h->count];
            it.a = dl[i];
            it.unit_begin = h->total;
            it.unit_off = parts[i].ddc_off;
            it.units = parts[i].ddc_cnt < 0 ? rfk::ddc_group_units(dl[i]) : parts[i].ddc_cnt;
            h->total += it.units;
            h->count++;
            dn[i].td = t;
        }
    }
    if (S->mode == RFS_MODE_GRAPH) {
        if (b.graph_version != S->class_version) {
            int rc = build_graph(S, b);
            if (rc) return rc;
        }
        if (hipGraphLaunch(b.exec, S->hs) != hipSuccess) return set_error(RF_EDEVICE, "hipGraphLaunch failed");
    } else {
        hipError_t e = hipMemcpyAsync(b.dev, b.host, S->region * NT, hipMemcpyHostToDevice, S->hs);
        if (e != hipSuccess) return set_error(RF_EDEVICE, "table upload failed");
        // the batch graph's topology, launched directly: table t on branch
        // t mod kMaxBranches (empty tables skipped), then join
        e = hipEventRecord(S->fork_ev[0], S->hs);
        int used = 0;
        for (int t = 0; t < NT && e == hipSuccess; ++t) {
            const rfk::GroupHeader *hh = hdr_at(b.host, S->region, t);
            if (hh->count == 0) continue;
            hipStream_t bs = S->branch[t % kMaxBranches];
            used = std::max(used, t % kMaxBranches + 1);
            e = hipStreamWaitEvent(bs, S->fork_ev[0], 0);
            if (e != hipSuccess) break;
            const rfk::GroupHeader *hd = hdr_at(b.dev, S->region, t);
            if (t < C) {
                const int grid = (int)std::min<int64_t>(hh->total, pfb_grid(S, S->classes[t].first));
                e = rfk::launch_pfb_group(S->classes[t].first, S->classes[t].second, hd,
                                          items_at<rfk::PfbItem>(b.dev, S->region, t), grid, bs);
            } else {
                const int grid = (int)std::min<int64_t>(hh->total, S->cus);
                e = rfk::launch_ddc_group(S->ddc_classes[t - C], hd, items_at<rfk::DdcItem>(b.dev, S->region, t),
                                          grid, bs);
            }
            if (e == hipSuccess) e = hipEventRecord(b.tev[t], bs);
        }
        for (int k = 0; k < used && e == hipSuccess; ++k) {
            e = hipEventRecord(S->fork_ev[1 + k], S->branch[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(S->hs, S->fork_ev[1 + k], 0);
        }
        if (e != hipSuccess) return set_error(RF_EDEVICE, "grouped launch failed");
    }
    for (size_t i = 0; i < who.size(); ++i) {
        Stream *s = who[i];
        if (!dn[i].req.n) continue;
        if (parts[i].pfb) rfi::pfb_commit(s->pfb, pl[i], dn[i].req.n, dn[i].pfb_frames, S->hs);
        if (s->ddc && parts[i].final) rfi::ddc_commit(s->ddc, dn[i].req.n, S->hs);
    }
    return RF_OK;
}

// Report one request's completion (caller holds mu).
void report(rfs_server *S, Done &d, double t)
{
    rfs_completion c{};
    c.stream = d.stream;
    c.slot = d.slot;
    c.tag = d.req.tag;
    c.nsamples = d.req.n;
    c.status = RF_OK;
    c.pfb_frames = d.pfb_frames;
    c.pfb_out = d.pfb_out;
    c.ddc_outputs = d.ddc_outputs;
    c.ddc_ld = d.ddc_ld;
    c.ddc_out = d.ddc_out;
    c.t_submit = d.req.t_submit;
    c.t_launch = d.t_launch;
    c.t_done = t;
    S->completions.push_back(c);
    auto it = S->streams.find(d.stream);
    if (it != S->streams.end()) {
        it->second->inflight--;
        if (d.stage >= 0) it->second->free_stage.push_back(d.stage);
    }
    S->st.requests++;
    S->st.samples += d.req.n;
    d.reported = true;
}

// Requests of a running grouped batch whose own kernels have finished.
void report_early(rfs_server *S, Blob &b)
{
    bool any = false;
    double t = 0;
    for (Done &d : b.done) {
        if (d.reported || d.partial || (d.tp < 0 && d.td < 0)) continue;
        if (d.tp >= 0 && hipEventQuery(b.tev[d.tp]) != hipSuccess) continue;
        if (d.td >= 0 && hipEventQuery(b.tev[d.td]) != hipSuccess) continue;
        if (!any) {
            t = now_s();
            any = true;
        }
        std::lock_guard<std::mutex> lk(S->mu);
        report(S, d, t);
    }
    if (any) S->cv_done.notify_all();
}

void finish_blob(rfs_server *S, Blob &b)
{
    const double t = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    for (Done &d : b.done)
        if (!d.reported && !d.partial) report(S, d, t);
    S->st.batches++;
    S->st.gpu_busy_seconds += t - b.t_launch;
    b.done.clear();
    b.busy = false;
    S->cv_done.notify_all();
}

void scheduler(rfs_server *S)
{
    (void)hipSetDevice(S->device);
    std::vector<Done> dn;
    std::vector<rfk::PfbLaunch> pl;
    std::vector<rfk::DdcLaunch> dl;
    std::vector<Stream *> who;
    std::vector<Part> parts;
    while (true) {
        // retire finished batches, oldest first
        for (int k = 0; k < 2; ++k) {
            Blob &b = S->blobs[(S->next_blob + k) & 1];
            if (!b.busy) continue;
            if (hipEventQuery(b.ev) == hipSuccess) finish_blob(S, b);
            else report_early(S, b);
        }
        Blob &b = S->blobs[S->next_blob];
        if (b.busy) {   // both blobs in flight: wait for the older one
            (void)hipEventSynchronize(b.ev);
            finish_blob(S, b);
        }
        dn.clear();
        pl.clear();
        dl.clear();
        who.clear();
        parts.clear();
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && S->blobs[0].busy == false && S->blobs[1].busy == false) {
                bool pending = false;
                for (auto &kv : S->streams) pending |= !kv.second->queue.empty() || kv.second->ch.on;
                if (!pending) break;
            }
            if (stage_copies(S)) {
                S->fatal = rf_last_error();
                S->stop = true;
                break;
            }
            if (!form_batch(S, dn, pl, dl, who, parts)) {
                const bool any_busy = S->blobs[0].busy || S->blobs[1].busy;
                if (S->stop && !any_busy) break;
                if (any_busy) {
                    lk.unlock();
                    std::this_thread::sleep_for(std::chrono::microseconds(20));
                } else {
                    S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                }
                continue;
            }
            int rc = launch_batch(S, b, dn, pl, dl, who, parts);
            if (rc) {
                S->fatal = rf_last_error();
                for (Stream *s : who) s->inflight--;
                S->stop = true;
                break;
            }
        }
        b.t_launch = now_s();
        for (Done &d : dn) d.t_launch = b.t_launch;
        b.done = dn;
        (void)hipEventRecord(b.ev, S->hs);
        b.busy = true;
        S->next_blob ^= 1;
    }
    for (int k = 0; k < 2; ++k)
        if (S->blobs[k].busy) {
            (void)hipEventSynchronize(S->blobs[k].ev);
            finish_blob(S, S->blobs[k]);
        }
}

}  // namespace

extern "C" {

double rfs_now(void) { return now_s(); }

uint64_t rfs_stream_footprint(const rfs_stream_desc *d) { return d ? footprint_of(d) : 0; }

int rfs_create(rfs_t *out, uint64_t hbm_budget_bytes, int32_t mode, int32_t max_streams)
{
    if (!out) return set_error(RF_EINVAL, "rfs_create: out is NULL");
    *out = nullptr;
    if (mode < RFS_MODE_SEQUENTIAL || mode > RFS_MODE_GRAPH) return set_error(RF_EINVAL, "rfs_create: bad mode");
    if (max_streams < 1 || max_streams > 4096) return set_error(RF_EINVAL, "rfs_create: max_streams out of range");
    rfs_server *S = new (std::nothrow) rfs_server;
    if (!S) return set_error(RF_ENOMEM, "rfs_create: host allocation");
    S->mode = mode;
    S->max_streams = max_streams;
    S->budget = hbm_budget_bytes;
    S->st.bytes_budget = hbm_budget_bytes;
    bool ok = hipGetDevice(&S->device) == hipSuccess;
    int cus = 0;
    if (ok && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device) == hipSuccess && cus > 0)
        S->cus = cus;
    ok = ok && hipStreamCreateWithFlags(&S->hs, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; ok && k < kMaxBranches; ++k) {
        hipStream_t bs = nullptr;
        ok = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking) == hipSuccess;
        if (ok) S->branch.push_back(bs);
    }
    for (int k = 0; ok && k < 1 + kMaxBranches; ++k) {
        hipEvent_t ev = nullptr;
        ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) S->fork_ev.push_back(ev);
    }
    // item tables sized for every open stream in up to max_streams PFB classes
    // and the five DDC work-group sizes
    S->region = region_bytes(max_streams);
    const size_t bytes = S->region * (size_t)(max_streams + 5);
    for (int k = 0; ok && k < 2; ++k) {
        Blob &b = S->blobs[k];
        b.bytes = bytes;
        ok = hipHostMalloc(&b.host, bytes, hipHostMallocDefault) == hipSuccess &&
             hipMalloc(&b.dev, bytes) == hipSuccess &&
             hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) == hipSuccess;
        for (int t = 0; ok && t < max_streams + 5; ++t) {
            hipEvent_t ev = nullptr;
            ok = hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
            if (ok) b.tev.push_back(ev);
        }
        if (ok) memset(b.host, 0, bytes);
    }
    if (!ok) {
        (void)hipGetLastError();
        rfs_destroy(S);
        return set_error(RF_EDEVICE, "rfs_create: HIP resource allocation failed");
    }
    S->thr = std::thread(scheduler, S);
    *out = S;
    return RF_OK;
}

int rfs_open_stream(rfs_t S, const rfs_stream_desc *d, int32_t *id)
{
    if (!S || !d || !id) return set_error(RF_EINVAL, "rfs_open_stream: NULL argument");
    *id = -1;
    if (!(d->kinds & (RFS_PFB | RFS_DDC)) || (d->kinds & ~(RFS_PFB | RFS_DDC)))
        return set_error(RF_EINVAL, "rfs_open_stream: kinds must be RFS_PFB and/or RFS_DDC");
    if (d->max_buffer < 1) return set_error(RF_EINVAL, "rfs_open_stream: max_buffer must be >= 1");
    if (d->host_slots < 0 || d->host_slots > 64) return set_error(RF_EINVAL, "rfs_open_stream: host_slots must be in [0, 64]");
    if ((d->kinds & RFS_PFB) && (d->nchan < 16 || d->nchan > 4096 || (d->nchan & (d->nchan - 1))))
        return set_error(RF_EINVAL, "rfs_open_stream: served PFB streams need a power-of-two nchan in [16, 4096]");
    const size_t fp = footprint_of(d);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if ((int)S->streams.size() >= S->max_streams)
            return set_error(RF_EAGAIN, "rfs_open_stream: max_streams are open");
        if (S->admitted + fp > S->budget)
            return set_error(RF_EAGAIN, "rfs_open_stream: footprint exceeds the remaining device-memory budget");
        S->admitted += fp;   // reserve
    }
    Stream *s = new (std::nothrow) Stream;
    int rc = s ? RF_OK : set_error(RF_ENOMEM, "rfs_open_stream: host allocation");
    if (!rc) {
        s->kinds = d->kinds;
        s->max_buffer = d->max_buffer;
        s->nslots = d->out_slots > 0 ? d->out_slots : 1;
        s->footprint = fp;
        if (d->kinds & RFS_PFB) {
            s->N = d->nchan;
            s->M = d->ntaps;
            rc = pfb_create(&s->pfb, d->nchan, d->ntaps, d->proto, RF_DFT_FFT_F32, d->max_buffer);
            s->pfb_cap = slot_frames(d->nchan, d->ntaps, d->max_buffer);
            for (int k = 0; !rc && k < s->nslots; ++k) {
                float *p = nullptr;
                if (hipMalloc((void **)&p, s->pfb_cap * d->nchan * 8) != hipSuccess)
                    rc = set_error(RF_ENOMEM, "rfs_open_stream: output slot allocation");
                else
                    s->pfb_slot.push_back(p);
            }
        }
        if (!rc && (d->kinds & RFS_DDC)) {
            s->ntones = d->ntones;
            rc = ddc_create(&s->ddc, d->ntones, d->phase_inc, d->phase0, d->lpf_taps, d->lpf, d->decim,
                            d->max_buffer);
            s->ddc_ld = slot_outputs(d->lpf_taps, d->decim, d->max_buffer);
            for (int k = 0; !rc && k < s->nslots; ++k) {
                float *p = nullptr;
                if (hipMalloc((void **)&p, (size_t)d->ntones * s->ddc_ld * 8) != hipSuccess)
                    rc = set_error(RF_ENOMEM, "rfs_open_stream: output slot allocation");
                else
                    s->ddc_slot.push_back(p);
            }
        }
        for (int k = 0; k < s->nslots; ++k) s->free_slots.push_back(s->nslots - 1 - k);
        for (int k = 0; !rc && k < d->host_slots; ++k) {
            uint32_t *p = nullptr;
            hipEvent_t ev = nullptr;
            if (hipMalloc((void **)&p, d->max_buffer * 4) != hipSuccess) {
                rc = set_error(RF_ENOMEM, "rfs_open_stream: staging slot allocation");
                break;
            }
            s->stage_buf.push_back(p);
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                rc = set_error(RF_EDEVICE, "rfs_open_stream: staging event");
                break;
            }
            s->stage_ev.push_back(ev);
            s->free_stage.push_back(d->host_slots - 1 - k);
        }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc) {
        S->admitted -= fp;
        free_stream(s);
        return rc;
    }
    s->id = S->next_id++;
    S->streams[s->id] = s;
    rebuild_classes(S);
    S->st.bytes_admitted = S->admitted;
    S->st.streams_open = (int)S->streams.size();
    *id = s->id;
    return RF_OK;
}

int rfs_submit(rfs_t S, int32_t id, const int16_t *iq, uint64_t nsamples, uint64_t tag)
{
    if (!S) return set_error(RF_EINVAL, "rfs_submit: server is NULL");
    bool host = false;
    if (nsamples > 0) {
        if (!iq || ((uintptr_t)iq & 3)) return set_error(RF_EINVAL, "rfs_submit: iq must be a non-NULL 4-byte aligned pointer");
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, iq) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(RF_EINVAL, "rfs_submit: iq is neither device memory nor pinned host memory");
        }
        if (at.type == hipMemoryTypeHost) host = true;
        else if (at.type != hipMemoryTypeDevice)
            return set_error(RF_EINVAL, "rfs_submit: iq is neither device memory nor pinned host memory");
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return set_error(RF_EDEVICE, S->fatal.empty() ? "rfs_submit: server stopped" : S->fatal.c_str());
    auto it = S->streams.find(id);
    if (it == S->streams.end() || it->second->closing) return set_error(RF_EINVAL, "rfs_submit: unknown stream");
    Stream *s = it->second;
    if (nsamples > s->max_buffer) return set_error(RF_EINVAL, "rfs_submit: nsamples exceeds the stream's max_buffer");
    if (host && s->stage_buf.empty())
        return set_error(RF_EINVAL, "rfs_submit: pinned-host buffer on a stream opened without host_slots");
    Request r{iq, nsamples, tag, now_s()};
    r.host = host;
    s->queue.push_back(r);
    S->cv_work.notify_one();
    return RF_OK;
}

int rfs_poll(rfs_t S, rfs_completion *out, int32_t max, int32_t *count, int32_t timeout_us)
{
    if (!S || !count || (max > 0 && !out)) return set_error(RF_EINVAL, "rfs_poll: NULL argument");
    *count = 0;
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->completions.empty() && timeout_us > 0)
        S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return !S->completions.empty(); });
    while (*count < max && !S->completions.empty()) {
        out[(*count)++] = S->completions.front();
        S->completions.pop_front();
    }
    if (*count == 0 && S->stop && !S->fatal.empty()) return set_error(RF_EDEVICE, S->fatal.c_str());
    return RF_OK;
}

int rfs_release(rfs_t S, int32_t id, int32_t slot)
{
    if (!S) return set_error(RF_EINVAL, "rfs_release: server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->streams.find(id);
    if (it == S->streams.end()) return set_error(RF_EINVAL, "rfs_release: unknown stream");
    Stream *s = it->second;
    if (slot < 0 || slot >= s->nslots ||
        std::find(s->free_slots.begin(), s->free_slots.end(), slot) != s->free_slots.end())
        return set_error(RF_EINVAL, "rfs_release: slot is not held");
    s->free_slots.push_back(slot);
    S->cv_work.notify_one();
    return RF_OK;
}

int rfs_close_stream(rfs_t S, int32_t id)
{
    if (!S) return set_error(RF_EINVAL, "rfs_close_stream: server is NULL");
    Stream *s = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->streams.find(id);
        if (it == S->streams.end()) return set_error(RF_EINVAL, "rfs_close_stream: unknown stream");
        if (!it->second->queue.empty() || it->second->inflight > 0)
            return set_error(RF_EAGAIN, "rfs_close_stream: the stream has queued or running requests");
        s = it->second;
        S->streams.erase(it);
        S->admitted -= s->footprint;
        rebuild_classes(S);
        S->st.bytes_admitted = S->admitted;
        S->st.streams_open = (int)S->streams.size();
    }
    free_stream(s);
    return RF_OK;
}

int rfs_get_stats(rfs_t S, rfs_stats *st)
{
    if (!S || !st) return set_error(RF_EINVAL, "rfs_get_stats: NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *st = S->st;
    return RF_OK;
}

int rfs_destroy(rfs_t S)
{
    if (!S) return RF_OK;
    if (S->thr.joinable()) {
        S->stop = true;
        S->cv_work.notify_all();
        S->thr.join();
    }
    if (S->hs) (void)hipStreamSynchronize(S->hs);
    if (S->cs) (void)hipStreamSynchronize(S->cs);
    for (auto &kv : S->streams) free_stream(kv.second);
    for (int k = 0; k < 2; ++k) {
        Blob &b = S->blobs[k];
        if (b.exec) (void)hipGraphExecDestroy(b.exec);
        if (b.graph) (void)hipGraphDestroy(b.graph);
        if (b.host) (void)hipHostFree(b.host);
        if (b.dev) (void)hipFree(b.dev);
        if (b.ev) (void)hipEventDestroy(b.ev);
        for (hipEvent_t e : b.tev) (void)hipEventDestroy(e);
    }
    for (hipEvent_t e : S->fork_ev) (void)hipEventDestroy(e);
    for (hipStream_t bs : S->branch) (void)hipStreamDestroy(bs);
    if (S->hs) (void)hipStreamDestroy(S->hs);
    if (S->cs) (void)hipStreamDestroy(S->cs);
    delete S;
    return RF_OK;
}

}  // extern "C"
