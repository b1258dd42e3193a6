// Kernel launchers of libcorr (internal; the public interface is corr.h).
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace corr {

struct FArgs;

// int8 MFMA X-engine; bt = 64 or 128; aligned: rows and base 16-byte aligned.
hipError_t launch_xeng_i8(const XArgs& a, int bt, bool aligned, hipStream_t s);
// Matrix-core X-engine for 16-byte aligned rows; elem = kElemI8 / kElemF16 / kElemF8
// (bt 64 or 128), or kElemCI4 / kElemF16Cvt / kElemF8Cvt (bt 128).
hipError_t launch_xeng_mfma(const XArgs& a, int elem, int bt, hipStream_t s);
// Serving grid over the device job queue (int8, aligned rows, 128-row tiles);
// grid = workgroups.
hipError_t launch_xeng_serve(const ServeQueue& q, int grid, hipStream_t s);
int serve_blocks_per_cu();
// FP32 X-engine; sample_bytes = 8 (complex float32) or 2 (complex int8).
hipError_t launch_xeng_f32(const XArgs& a, int sample_bytes, int bt, bool aligned, hipStream_t s);
hipError_t launch_reduce_splits(const void* part, int64_t n_pairs, int n_split, void* acc, int accumulate,
                                bool is_int, hipStream_t s);
hipError_t launch_fold_f64(double* L, const void* V, int64_t n_scalars, bool is_int, hipStream_t s);
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s);   // 16-byte aligned, bytes / 16 words
hipError_t launch_fill_zero_bytes(void* p, int64_t bytes, hipStream_t s);

// Guard bands of a plan's workspace: kGuardBytes after each region, filled
// with a pattern that depends on the band and the word, and compared later.
constexpr int kGuardBytes = 256;
constexpr int kMaxGuards = 12;
struct GuardList {
  uint64_t off[kMaxGuards];   // byte offsets of the bands in the workspace (256-byte aligned)
  int32_t n;
};
hipError_t launch_guard_fill(uint8_t* ws, const GuardList& g, hipStream_t s);
// Writes the number of guard words that differ from the pattern to *bad.
hipError_t launch_guard_check(const uint8_t* ws, const GuardList& g, uint32_t* bad, hipStream_t s);

struct FStageCall {
  const void* volt;        // real int8 (format 0), 16-bit 5+5 words (1) or 4+4 bytes (2)
  const float2* twiddle;
  int8_t* ring;
  float* dbg;
  int64_t n_blocks;
  int64_t ring_stride;
  int64_t t_offset;
  int32_t n_in;
  float scale;
  float max_abs;
  int32_t format;          // 0: real 256-point F-stage; 1, 2: complex 128-point F-stage
  int32_t pfb_taps;        // real F-stage: > 1 = polyphase filterbank taps (volt holds taps - 1 more blocks)
  const float* pfb;        // filterbank coefficients [pfb_taps * 256]
};
hipError_t launch_fstage_call(const FStageCall& c, hipStream_t s);
hipError_t launch_fstage_complex(const FStageCall& c, hipStream_t s);
hipError_t launch_cmac_design(int design, int group, const float2* x, int64_t T, int n_in, int n_ch, float2* out,
                              int accumulate, hipStream_t s);
hipError_t launch_aggregate_w16(const uint16_t* rec, int32_t n_streams, int32_t w_per, int64_t n_rec,
                                uint32_t first_counter, uint16_t* out, uint32_t* bad, hipStream_t s);

struct LowpCall {
  const float* x;          // complex float32 [n_ch][n_in][row_stride]
  int64_t n_ch;
  int64_t n_in;
  int64_t n_t;             // samples converted per row
  int64_t row_stride;      // input samples per row
  int64_t out_stride;      // staged samples per row
  int elem;                // kElemF16 or kElemF8
  void* out;               // staged [n_ch][n_in][out_stride] (re, im) elements
  uint32_t* m_bits;        // FP8: per-channel max |x| (float bits), scratch
  float* inv_scale2;       // FP8: per-channel 1/s_c^2 (output)
};
hipError_t launch_lowp_stage(const LowpCall& c, hipStream_t s);
// Per-channel max |re|, |im| (float bits) of complex float32 [n_ch][n_in][row_stride] rows.
hipError_t launch_absmax(const float* x, int64_t n_ch, int64_t n_in, int64_t n_t, int64_t row_stride, uint32_t* m_bits,
                         hipStream_t s);

}  // namespace corr
