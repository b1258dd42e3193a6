// Internal plan helpers shared by the serving scheduler (not part of the C ABI).
#pragma once

#include "corr.h"

// Queue the integration read-out of `p` into `dst` (device memory if
// dst_is_device, else host) on the plan's stream without synchronising, then
// reset the accumulator (the asynchronous form of corr_dump(CORR_DUMP_INTEG)).
// *n_samples_out receives the sample count of the integration.
extern "C" __attribute__((visibility("hidden"))) corr_status corr_internal_dump_async(corr_plan* p, void* dst,
                                                                                        int32_t dst_is_device,
                                                                                        int64_t* n_samples_out);
