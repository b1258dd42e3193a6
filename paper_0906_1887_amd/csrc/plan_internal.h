// Internal plan helpers shared by the translation units of libcorr (not part
// of the C ABI; hidden from the library's exported symbols).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "corr.h"

#define CORR_HIDDEN __attribute__((visibility("hidden")))

// Queue the integration read-out of `p` into `dst` (device memory if
// dst_is_device, else host) on the plan's stream without synchronising, then
// reset the accumulator (the asynchronous form of corr_dump(CORR_DUMP_INTEG)).
// *n_samples_out receives the sample count of the integration.
extern "C" CORR_HIDDEN corr_status corr_internal_dump_async(corr_plan* p, void* dst, int32_t dst_is_device,
                                                            int64_t* n_samples_out);

// One X-engine pass with every device buffer explicit: samples x
// [n_ch][n_in][row_stride] (sb bytes per sample; elem >= 0 selects the staged
// FP16/FP8 matrix-core engine; kElemF16Cvt / kElemF8Cvt read CF32 rows)
// added to (accumulate) or stored into acc
// [n_ch][P][2].  part: K-split partials (split * acc bytes), only needed when
// corr_internal_split > 1; a reduction kernel then adds them into acc in split
// order.  m_bits: the converting FP8 engine's per-channel maxima.
struct corr_xpass {
  const corr_config* cfg;
  const void* x;
  int sb;
  int elem;
  int64_t n_samples;
  int64_t row_stride;
  const float* inv_scale2;
  const uint32_t* m_bits;   // converting FP8 engine: per-channel max |re|, |im|
  void* acc;
  int accumulate;
  void* part;
  size_t part_bytes;
  hipStream_t stream;
};
CORR_HIDDEN corr_status corr_internal_xengine(const corr_xpass* q);
// K splits of a pass of n_samples for configuration c (1 = no partials).
CORR_HIDDEN int corr_internal_split(const corr_config* c, int64_t n_samples);
