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
constexpr int kElemCI4 = 3;   // int8 engine on 4-bit complex samples, one byte each

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

// Team schedule of the 128-row int8 engine (xeng_team_kernel).  Sync words
// (uint32, zero at launch): per XCD, one per team plus the diagonal-tile
// queue, each on its own 128-byte line.
constexpr int kTeamSyncLine = 32;                  // uint32 per line
constexpr int kTeamSyncStride = 4 * kTeamSyncLine; // per XCD: up to 3 teams + queue
struct TeamArgs {
  XArgs x;
  uint32_t* sync;           // [kNumXcd][kTeamSyncStride]
  int32_t nb;               // row panels of 128 inputs
  int32_t n_full;           // off-diagonal tiles per channel = workgroups per team
  int32_t teams;            // teams per XCD (1..3)
  int32_t slack;            // steps a member may start ahead of its team's slowest
  int32_t spin_limit;       // polls before a member stops waiting
  int32_t pad_;
};

// Serving queue (xeng_serve_kernel).  The host publishes each admitted job
// in a slot; the claim and done words of a slot count items over all the jobs
// the slot has held and are never reset, so a job's items are the claim
// values [base, base + n_items).
constexpr int kServeLine = 32;             // uint32 per 128-byte line
constexpr int kServeSmall = 1 << 16;       // active-list flag: the slot's job has 64-row tiles
struct ServeJob {
  XArgs x;                  // the job's pass: samples, strides, output, n_tiles, n_items (channel x tile)
  uint32_t* flag;           // completion word in host memory (device view)
  uint32_t flag_value;      // written there when the job's last item is done
  int32_t bt;               // tile rows: 64 or 128
  uint64_t base;            // claim value of the job's first item
  uint64_t pad_[3];
};
struct ServeQueue {
  const ServeJob* slots;    // [n_slots]
  const uint64_t* limit;    // slot s at limit[s * kServeLine / 2]: base + n_items of its job
  uint64_t* claim;          // slot s at claim[s * kServeLine / 2]
  uint32_t* done;           // slot s at done[s * kServeLine]
  const int32_t* active;    // [1 + n_slots]: count, then the slots holding jobs
                            // (| kServeSmall for 64-row jobs)
  uint32_t* rr;             // round-robin counter
  int32_t n_slots;
  int32_t idle_polls;       // polls without work before a workgroup exits
};

}  // namespace corr
