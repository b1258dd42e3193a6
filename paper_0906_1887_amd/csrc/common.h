// Internal helpers shared by the libcorr kernels and host code (not part of
// the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace corr {

// Workgroups are handed to the 8 XCDs of an MI355X round-robin by workgroup
// id, and each XCD has its own L2.  Kernels remap blockIdx.x so that a
// contiguous range of work items (e.g. all baseline tiles of one channel,
// which re-read the same input rows) runs on one XCD, in order.
constexpr int kNumXcd = 8;

// Element kinds of the matrix-core X-engine.
constexpr int kElemI8 = 0;
constexpr int kElemF16 = 1;
constexpr int kElemF8 = 2;

__device__ __forceinline__ int64_t xcd_item(int64_t bid, int64_t per_xcd) {
  const int64_t xcd = bid % kNumXcd;
  const int64_t slot = bid / kNumXcd;
  return xcd * per_xcd + slot;
}

// Lower-triangle tile (I >= J) of linear index t = I(I+1)/2 + J.
__device__ __forceinline__ void tile_decode(int t, int& I, int& J) {
  int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
  while (i * (i + 1) / 2 > t) --i;
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  I = i;
  J = t - i * (i + 1) / 2;
}

__device__ __forceinline__ int64_t tri_index(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

// Kernel argument block of the X-engines.
struct XArgs {
  const void* x;            // samples [n_ch][n_in][row_stride] (complex)
  int64_t row_stride_b;     // bytes between consecutive input rows
  int64_t ch_stride_b;      // bytes between channels
  int64_t k_bytes;          // valid bytes per row (n_samples * bytes per sample)
  int64_t k_split_bytes;    // bytes per K split (multiple of the K chunk)
  void* out;                // accumulator [n_ch][P][2] (or split partials)
  int64_t out_split_stride; // elements between split partial buffers
  int64_t n_products;       // P
  int32_t n_in;
  int32_t n_ch;
  int32_t n_tiles;          // lower-triangle tiles per channel
  int32_t n_split;          // K splits
  int32_t n_items;          // n_ch * n_tiles * n_split
  int32_t per_xcd;          // ceil(n_items / 8)
  int32_t accumulate;       // 1: out += tile; 0: out = tile
  int32_t pad_;
  const float* inv_scale2;  // FP8: per-channel 1/s_c^2 applied in the epilogue (else null)
};

}  // namespace corr
