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
constexpr int kElemF16Cvt = 4;  // FP16 engine converting complex float32 as it stages
constexpr int kElemF8Cvt = 5;   // FP8 engine converting (with the per-channel scale) as it stages
constexpr int kElemF32 = 6;     // complex float32 on v_mfma_f32_16x16x4_f32 (64-row tiles)

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
  const uint32_t* m_bits;   // converting FP8 engine: per-channel max |re|, |im| (float bits)
};

// Work item -> (channel, K split, tile I >= J) of the matrix-core engines:
// tile fastest, then split, then channel, so that a channel's tiles (which
// share its row panels) start together on one XCD (xcd_item keeps each XCD's
// items contiguous).  An order that ran each XCD's off-diagonal tiles before
// its diagonal ones read less from HBM on C3 but was measured slower there
// (1.5 %) and on the FP16 engine (10 %), so it was removed.
__device__ __forceinline__ void item_decode(const XArgs& a, int64_t item, int& ch, int& split, int& I, int& J) {
  const int tile = (int)(item % a.n_tiles);
  const int64_t rest = item / a.n_tiles;
  split = (int)(rest % a.n_split);
  ch = (int)(rest / a.n_split);
  tile_decode(tile, I, J);
}

// FP8 scale of a channel with max |re|, |im| = m: the largest power of two s
// with s * m <= 448 (the largest finite E4M3 value); 1 when m is 0 or not
// finite.  The exponent is kept in [-60, 60] (so 1/s^2 stays a normal float)
// and the correction loops are bounded; within that range the result is
// exact, because s is a power of two and the comparisons are exact.
__device__ __forceinline__ float e4m3_scale(float m) {
  if (!(m > 0.f) || !(m < INFINITY)) return 1.f;
  const float e = fminf(fmaxf(floorf(log2f(448.f / m)), -60.f), 60.f);
  float s = ldexpf(1.f, (int)e);
  for (int k = 0; k < 4 && s * m > 448.f && s > 0x1p-60f; ++k) s *= 0.5f;
  for (int k = 0; k < 4 && 2.f * s * m <= 448.f && s < 0x1p60f; ++k) s *= 2.f;
  return s;
}

// Serving queue (xeng_serve_kernel).  The host publishes each admitted job
// in a slot; the claim and done words of a slot count items over all the jobs
// the slot has held and are never reset, so a job's items are the claim
// values [base, base + n_items).  Every job runs 128-row tiles.
constexpr int kServeLine = 32;             // uint32 per 128-byte line
struct ServeJob {
  XArgs x;                  // the job's pass: samples, strides, output, n_tiles, n_items (channel x tile)
  uint32_t* flag;           // completion word in host memory (device view)
  uint32_t flag_value;      // written there when the job's last item is done
  int32_t pad0_;
  uint64_t base;            // claim value of the job's first item
  uint64_t pad_[3];
};
struct ServeQueue {
  const ServeJob* slots;    // [n_slots]
  const uint64_t* limit;    // slot s at limit[s * kServeLine / 2]: base + n_items of its job
  uint64_t* claim;          // slot s at claim[s * kServeLine / 2]
  uint32_t* done;           // slot s at done[s * kServeLine]
  const int32_t* active;    // [1 + n_slots]: count, then the slots whose jobs have unclaimed items
  uint32_t* rr;             // round-robin counter
  uint64_t* last_claim;     // wall clock (s_memrealtime ticks) of the latest claim or grid start
  uint32_t* closing;        // highest grid generation that has closed (no more claims)
  uint32_t* host_closing;   // the same, in host memory (device view) for the scheduler
  uint64_t* host_claimed;   // host memory (device view): slot s at [s * kServeLine / 2 + 1] receives
                            // the claim limit of its job once the job's last item is claimed
  uint32_t gen;             // this launch's generation (increasing from 1)
  uint32_t idle_ticks;      // queue idle this long (100 MHz ticks): the grid closes
  int32_t n_slots;
  int32_t max_polls;        // bound on one workgroup's empty polls (a safety net)
};

}  // namespace corr
