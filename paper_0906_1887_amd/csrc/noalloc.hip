// corr_correlate_static: the X-engine pass of corr_correlate for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  It runs the same kernels; the
// buffer that corr_correlate takes from the plan's workspace -- the K-split
// partial tiles -- comes from `scratch`, a fixed
// array in the library's device image, and the accumulator is the caller's
// output buffer.  It calls no hipMalloc, hipFree or allocating
// library routine.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "common.h"
#include "corr.h"
#include "launch.h"
#include "plan_internal.h"

namespace {

constexpr size_t kScratchBytes = CORR_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

// One copy per GPU, held until the process ends.  In host code this name is
// only a handle for hipGetSymbolAddress: the device address is taken once per
// device and only that address is passed to kernels and fills.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

struct DeviceScratch {
  std::once_flag once;
  void* ptr = nullptr;
  hipError_t err = hipSuccess;
};
DeviceScratch g_scratch[kMaxDevices];

// Device address of the current device's scratch (looked up on the first call
// on that device, with that device current), or nullptr on failure.
void* scratch_ptr(hipError_t* err) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    *err = e != hipSuccess ? e : hipErrorInvalidDevice;
    return nullptr;
  }
  DeviceScratch& d = g_scratch[dev];
  std::call_once(d.once, [&d]() { d.err = hipGetSymbolAddress(&d.ptr, HIP_SYMBOL(scratch)); });
  *err = d.err;
  return d.err == hipSuccess ? d.ptr : nullptr;
}

}  // namespace

extern "C" corr_status corr_correlate_static(const corr_config* cfg, const void* d_samples, int64_t n_samples,
                                             int64_t row_stride, void* d_out, int32_t accumulate,
                                             void* hip_stream) {
  try {
    if (!cfg || !d_out || n_samples < 0 || row_stride < 0) return CORR_E_INVAL;
    size_t ws = 0;
    const corr_status v = corr_workspace_bytes(cfg, &ws);   // validates the configuration
    if (v != CORR_OK) return v;
    if (cfg->fft_size != 0 || cfg->fp64_longrun != 0) return CORR_E_INVAL;
    if (cfg->engine != CORR_X_I8 && cfg->engine != CORR_X_FP32) return CORR_E_UNSUPPORTED;
    if (n_samples > 0 && !d_samples) return CORR_E_INVAL;
    const int64_t stride = row_stride == 0 ? n_samples : row_stride;
    if (stride < n_samples) return CORR_E_INVAL;
    const bool ci4 = cfg->sample_type == CORR_CI4;
    const int sb = cfg->sample_type == CORR_CI8 ? 2 : (ci4 ? 1 : 8);
    if ((reinterpret_cast<uintptr_t>(d_samples) % (sb == 8 ? 4 : sb)) != 0) return CORR_E_INVAL;
    if (ci4 && n_samples > 0 && ((reinterpret_cast<uintptr_t>(d_samples) % 16) != 0 || stride % 16 != 0))
      return CORR_E_UNSUPPORTED;
    if (cfg->max_abs > 0) {
      const double bound = 2.0 * cfg->max_abs * cfg->max_abs * (double)n_samples * (ci4 ? 256.0 : 1.0);
      if (cfg->engine == CORR_X_I8 && bound > 2147483647.0) return CORR_E_OVERFLOW;
      if (cfg->engine == CORR_X_FP32 && bound > 16777216.0) return CORR_E_OVERFLOW;
    }
    if (n_samples == 0) return CORR_OK;

    // Scratch: the K-split partial tiles (none without a split).  Every
    // partial element is written by the pass before the reduction reads it,
    // so nothing needs clearing between calls.
    const int64_t P = (int64_t)cfg->n_inputs * (cfg->n_inputs + 1) / 2;
    const size_t acc_bytes = (size_t)cfg->n_channels * (size_t)P * 8;
    const int split = corr_internal_split(cfg, n_samples);
    const size_t part_bytes = split > 1 ? (size_t)split * acc_bytes : 0;
    if (part_bytes > kScratchBytes) return CORR_E_WORKSPACE;

    hipError_t e = hipSuccess;
    uint8_t* base = static_cast<uint8_t*>(scratch_ptr(&e));
    if (!base) return CORR_E_HIP;

    corr_xpass q;
    std::memset(&q, 0, sizeof(q));
    q.cfg = cfg;
    q.x = d_samples;
    q.sb = sb;
    q.elem = ci4 ? corr::kElemCI4 : -1;
    q.n_samples = n_samples;
    q.row_stride = stride;
    q.acc = d_out;
    q.accumulate = accumulate ? 1 : 0;
    q.part = part_bytes ? base : nullptr;
    q.part_bytes = part_bytes;
    q.stream = static_cast<hipStream_t>(hip_stream);
    return corr_internal_xengine(&q);
  } catch (...) {
    return CORR_E_INVAL;
  }
}
