// rf_handles.hpp -- internal split of the process calls, shared with the
// serving core: prepare() validates a call and fills the kernel arguments from
// the handle's host state without launching; commit() advances the handle's
// state once the launch has been enqueued.
#pragma once
#include <stddef.h>

#include "../../include/rfchan.h"
#include "rf_internal.hpp"

struct rf_pfb;
struct rf_ddc;

namespace rfi {

int pfb_prepare(rf_pfb *p, const int16_t *iq_dev, uint64_t nsamples, float *out_dev, uint64_t out_cap_frames,
                rfk::PfbLaunch *a, uint64_t *frames);
void pfb_commit(rf_pfb *p, const rfk::PfbLaunch &a, uint64_t nsamples, uint64_t frames, hipStream_t s);
int pfb_device(const rf_pfb *p);
int pfb_mode(const rf_pfb *p);
size_t pfb_footprint(int N, int M, int mode);

int ddc_prepare(rf_ddc *p, const int16_t *iq_dev, uint64_t nsamples, float *out_dev, uint64_t ld,
                rfk::DdcLaunch *a, uint64_t *nout);
void ddc_commit(rf_ddc *p, uint64_t nsamples, hipStream_t s);
int ddc_device(const rf_ddc *p);
int ddc_ntones(const rf_ddc *p);
size_t ddc_footprint(int ntones, int T);

// Last-error plumbing of the C ABI (thread-local message).
int set_error(int status, const char *msg);

}  // namespace rfi
