// libcorr host side: the C ABI declared in include/corr.h.
//
// Plan = validated configuration + views into the caller's workspace:
//   acc      integration accumulator [n_ch][P][2] (int32 for the int8 engine,
//            float32 otherwise); "logically zero" after a reset, so the next
//            X-engine pass stores instead of read-modify-writing
//   longrun  FP64 long-run accumulator [n_ch][P][2] (optional)
//   ring     F-stage output [n_ch][n_in][ring_stride] complex int8 (optional)
//   part     K-split partial tiles [max_split][n_ch][P][2] (small N_I only)
//   twiddle  W_256^m table for the F-stage (optional)
// The library never allocates device memory.
#include "corr.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "launch.h"
#include "plan_internal.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kSplitGranule = 64;  // samples; multiple of every engine's K chunk
constexpr int kMaxSplit = 16;
constexpr int kTargetItems = 1024;     // workgroups wanted per X-engine launch (split-K below this)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
  size_t acc = 0, acc_bytes = 0;
  size_t longrun = 0, longrun_bytes = 0;
  size_t ring = 0, ring_bytes = 0;
  size_t part = 0, part_bytes = 0;
  size_t tw = 0, tw_bytes = 0;
  size_t pfb = 0, pfb_bytes = 0;       // filterbank coefficients (pfb_taps > 1)
  size_t stage = 0, stage_bytes = 0;   // FP16/FP8 staged samples
  size_t mbits = 0, scales = 0;        // FP8 per-channel max and 1/s^2
  int64_t stage_stride = 0;            // staged samples per row
  int stage_sb = 0;                    // staged bytes per complex sample
  size_t total = 0;
  int max_split = 1;
  int bt = 128;
  int n_tiles = 0;
  int64_t ring_stride = 0;
  int64_t n_products = 0;
  corr::GuardList guards{};            // a guard band after each region
  size_t status = 0;                   // 256 bytes: the guard check's result word
};

int64_t n_products(int64_t n) { return n * (n + 1) / 2; }

corr_status validate(const corr_config* c) {
  if (!c) return CORR_E_INVAL;
  if (c->n_inputs < 1 || c->n_inputs > 65536 || c->n_channels < 1) return CORR_E_INVAL;
  if (c->engine < CORR_X_FP32 || c->engine > CORR_X_FP32M) return CORR_E_INVAL;
  if (c->sample_type != CORR_CF32 && c->sample_type != CORR_CI8 && c->sample_type != CORR_CI4) return CORR_E_INVAL;
  if (c->sample_type == CORR_CI4) {
    // nibble samples: int8 engine, |re|, |im| <= 7, X-engine input only
    if (c->max_abs < 1 || c->max_abs > 7 || c->fft_size != 0) return CORR_E_INVAL;
    if (c->engine != CORR_X_I8) return CORR_E_UNSUPPORTED;
  }
  if (c->max_abs < 0 || c->max_abs > 127) return CORR_E_INVAL;
  if (c->engine == CORR_X_F16 || c->engine == CORR_X_F8) {
    // float samples staged to FP16 / FP8 in chunks of ring_samples
    if (c->sample_type != CORR_CF32 || c->max_abs != 0 || c->fft_size != 0) return CORR_E_INVAL;
    if (c->ring_samples < 0) return CORR_E_INVAL;   // 0: convert while staging, no chunked staging buffer
    if (c->n_channels > 65535 || c->n_inputs > 65535) return CORR_E_UNSUPPORTED;
  }
  if (c->engine == CORR_X_FP32M) {
    // complex float32 samples straight into the FP32 matrix cores
    if (c->sample_type != CORR_CF32 || c->fft_size != 0) return CORR_E_INVAL;
  }
  if (c->engine == CORR_X_I8) {
    if (c->sample_type == CORR_CF32 && c->fft_size == 0) return CORR_E_INVAL;
    if (c->max_abs < 1) return CORR_E_INVAL;  // int32 bound needs a declared range
  }
  if (c->pfb_taps < 0) return CORR_E_INVAL;
  if (c->fft_size == 0 && (c->volt_format != CORR_VOLT_R8 || c->pfb_taps != 0)) return CORR_E_INVAL;
  if (c->pfb_taps > 1 && c->volt_format != CORR_VOLT_R8) return CORR_E_UNSUPPORTED;
  if (c->pfb_taps > 1 && c->pfb_taps != 4) return CORR_E_UNSUPPORTED;
  if (c->fft_size != 0) {
    if (c->volt_format == CORR_VOLT_R8) {
      if (c->fft_size != 2 * c->n_channels) return CORR_E_INVAL;
      if (c->fft_size != 256) return CORR_E_UNSUPPORTED;
    } else if (c->volt_format == CORR_VOLT_CW16 || c->volt_format == CORR_VOLT_CB8) {
      if (c->fft_size != c->n_channels) return CORR_E_INVAL;
      if (c->fft_size != 128) return CORR_E_UNSUPPORTED;
    } else {
      return CORR_E_INVAL;
    }
    if (c->max_abs < 1) return CORR_E_INVAL;
    if (!(c->requant_scale > 0.0f) || !std::isfinite(c->requant_scale)) return CORR_E_INVAL;
    if (c->ring_samples < 1) return CORR_E_INVAL;
  }
  if (c->ring_samples < 0) return CORR_E_INVAL;
  return CORR_OK;
}

Layout layout_of(const corr_config* c) {
  Layout L;
  L.n_products = n_products(c->n_inputs);
  // CI4 and the converting FP16/FP8 engines run 128-row tiles only
  const bool lowp_cvt = (c->engine == CORR_X_F16 || c->engine == CORR_X_F8) && c->ring_samples == 0;
  // the FP32 matrix-core engine runs 64-row tiles only
  L.bt = c->engine != CORR_X_FP32M && (c->n_inputs > 64 || c->sample_type == CORR_CI4 || lowp_cvt) ? 128 : 64;
  const int64_t nb = (c->n_inputs + L.bt - 1) / L.bt;
  L.n_tiles = (int)(nb * (nb + 1) / 2);
  const int64_t tiles_total = (int64_t)c->n_channels * L.n_tiles;
  L.max_split = tiles_total >= kTargetItems
                    ? 1
                    : (int)std::min<int64_t>(kMaxSplit, (kTargetItems + tiles_total - 1) / tiles_total);
  const size_t pair_bytes = 8;  // int2 (int8 engine) or float2 (others)
  size_t off = 0;
  // each region is followed by a guard band (checked by corr_dump)
  auto end_region = [&](size_t bytes) {   // at most 9 regions, below kMaxGuards
    off = align_up(off + bytes, kAlign);
    if (L.guards.n < corr::kMaxGuards) L.guards.off[L.guards.n++] = off;
    off += corr::kGuardBytes;
  };
  L.acc = off;
  L.acc_bytes = (size_t)c->n_channels * L.n_products * pair_bytes;
  end_region(L.acc_bytes);
  if (c->fp64_longrun) {
    L.longrun = off;
    L.longrun_bytes = (size_t)c->n_channels * L.n_products * 16;
    end_region(L.longrun_bytes);
  }
  if (c->fft_size != 0) {
    L.ring_stride = (c->ring_samples + 63) / 64 * 64;
    L.ring = off;
    L.ring_bytes = (size_t)c->n_channels * c->n_inputs * L.ring_stride * 2;
    end_region(L.ring_bytes);
    L.tw = off;
    L.tw_bytes = (size_t)c->fft_size * sizeof(float2);
    end_region(L.tw_bytes);
    if (c->pfb_taps > 1) {
      L.pfb = off;
      L.pfb_bytes = (size_t)c->pfb_taps * c->fft_size * sizeof(float);
      end_region(L.pfb_bytes);
    }
  }
  if (c->engine == CORR_X_F16 || c->engine == CORR_X_F8) {
    L.stage_sb = (c->engine == CORR_X_F16) ? 4 : 2;
    L.stage_stride = (c->ring_samples + 63) / 64 * 64;
    L.stage = off;
    L.stage_bytes = (size_t)c->n_channels * c->n_inputs * L.stage_stride * L.stage_sb;   // 0 when converting
    end_region(L.stage_bytes);
    L.mbits = off;
    end_region((size_t)c->n_channels * 4);
    L.scales = off;
    end_region((size_t)c->n_channels * 4);
  }
  if (L.max_split > 1) {
    L.part = off;
    L.part_bytes = (size_t)L.max_split * L.acc_bytes;
    end_region(L.part_bytes);
  }
  L.status = off;
  L.total = off + kAlign;
  return L;
}

}  // namespace

struct corr_plan {
  corr_config cfg;
  Layout L;
  hipStream_t stream;
  uint8_t* ws;
  std::vector<float2> tw_host;
  std::vector<float> pfb_host;   // filterbank coefficients (kept for the asynchronous upload)
  int64_t n_accum = 0;       // samples in the integration accumulator
  int64_t n_long = 0;        // samples folded into the FP64 long-run accumulator
  bool acc_zero = true;      // accumulator logically zero (contents stale)
  bool error = false;
  bool seq_valid = false;
  bool guards_set = false;   // the workspace's guard bands hold their pattern
  uint64_t next_seq = 0;
  int64_t ring_fill = 0;     // samples waiting in the ring
  int64_t stage_fill = 0;    // samples of the last FP16/FP8 staged chunk
};

namespace {

corr_status hip_fail(corr_plan* p, hipError_t e) {
  if (e == hipSuccess) return CORR_OK;
  p->error = true;
  return CORR_E_HIP;
}

void* at(corr_plan* p, size_t off) { return p->ws + off; }

// Fill the guard bands before the plan's first kernel writes its workspace.
hipError_t ensure_guards(corr_plan* p) {
  if (p->guards_set) return hipSuccess;
  const hipError_t e = corr::launch_guard_fill(p->ws, p->L.guards, p->stream);
  if (e == hipSuccess) p->guards_set = true;
  return e;
}

// Launch one X-engine pass over samples [n_ch][n_in][row_stride] (bytes per
// sample `sb`), n_samples per row, into the plan's accumulator.
corr_status xengine_pass(corr_plan* p, const void* x, int sb, int64_t n_samples, int64_t row_stride,
                         int elem = -1, const float* inv_scale2 = nullptr, const uint32_t* m_bits = nullptr) {
  const Layout& L = p->L;
  corr_xpass q;
  std::memset(&q, 0, sizeof(q));
  q.cfg = &p->cfg;
  q.x = x;
  q.sb = sb;
  q.n_samples = n_samples;
  q.row_stride = row_stride;
  q.elem = elem;
  q.inv_scale2 = inv_scale2;
  q.m_bits = m_bits;
  q.acc = at(p, L.acc);
  q.accumulate = p->acc_zero ? 0 : 1;
  q.part = L.part_bytes ? at(p, L.part) : nullptr;
  q.part_bytes = L.part_bytes;
  q.stream = p->stream;
  const corr_status st = corr_internal_xengine(&q);
  if (st == CORR_E_HIP) p->error = true;
  if (st == CORR_OK && n_samples > 0) p->acc_zero = false;
  return st;
}

}  // namespace

int corr_internal_split(const corr_config* c, int64_t n_samples) {
  const Layout L = layout_of(c);
  const int64_t n_gran = (n_samples + kSplitGranule - 1) / kSplitGranule;
  // At least two granules (128 samples) per split: a 1000-sample integration
  // at N_I = 64 then takes 8 splits, 3 % faster than 4 splits of 256.
  int split = (int)std::min<int64_t>(L.max_split, std::max<int64_t>(1, n_gran / 2));
  const int64_t gran_per_split = (n_gran + split - 1) / split;
  return (int)((n_gran + gran_per_split - 1) / gran_per_split);
}

corr_status corr_internal_xengine(const corr_xpass* q) {
  const corr_config& c = *q->cfg;
  const Layout L = layout_of(&c);
  const int64_t n_samples = q->n_samples;
  const int sb = q->sb;
  if (n_samples == 0) return CORR_OK;
  const int64_t n_gran = (n_samples + kSplitGranule - 1) / kSplitGranule;
  const int split = corr_internal_split(&c, n_samples);
  const int64_t gran_per_split = (n_gran + split - 1) / split;
  if (split > 1 && (!q->part || q->part_bytes < (size_t)split * L.acc_bytes)) return CORR_E_WORKSPACE;

  corr::XArgs a;
  std::memset(&a, 0, sizeof(a));
  a.x = q->x;
  // converting engines read float32 rows (8 bytes per sample); their K
  // counts staged bytes (sb per sample)
  const bool cvt = q->elem == corr::kElemF16Cvt || q->elem == corr::kElemF8Cvt;
  a.row_stride_b = q->row_stride * (cvt ? 8 : sb);
  a.ch_stride_b = (int64_t)c.n_inputs * a.row_stride_b;
  a.k_bytes = n_samples * sb;
  a.k_split_bytes = gran_per_split * kSplitGranule * sb;
  a.n_products = L.n_products;
  a.n_in = c.n_inputs;
  a.n_ch = c.n_channels;
  a.n_tiles = L.n_tiles;
  a.n_split = split;
  const int64_t items = (int64_t)c.n_channels * L.n_tiles * split;
  if (items > 0x7FFFFFFFll / 2) return CORR_E_INVAL;
  a.n_items = (int32_t)items;
  a.per_xcd = (int32_t)((items + corr::kNumXcd - 1) / corr::kNumXcd);
  const bool direct = (split == 1);
  a.out = direct ? q->acc : q->part;
  a.out_split_stride = direct ? 0 : (int64_t)c.n_channels * L.n_products;
  a.accumulate = direct ? q->accumulate : 0;
  a.inv_scale2 = q->inv_scale2;
  a.m_bits = q->m_bits;
  const bool aligned = (a.row_stride_b % 16 == 0) && ((reinterpret_cast<uintptr_t>(q->x) & 15) == 0);
  // nibble rows and FP32 matrix-core rows are staged 16 bytes at a time
  if ((q->elem == corr::kElemCI4 || q->elem == corr::kElemF32) && !aligned) return CORR_E_UNSUPPORTED;

  hipError_t e;
  const bool is_int = (c.engine == CORR_X_I8);
  if (q->elem >= 0)
    e = corr::launch_xeng_mfma(a, q->elem, L.bt, q->stream);  // staged FP16 / FP8 rows and CI4 rows are aligned
  else if (c.engine == CORR_X_I8)
    e = aligned ? corr::launch_xeng_mfma(a, corr::kElemI8, L.bt, q->stream)
                : corr::launch_xeng_i8(a, L.bt, false, q->stream);
  else
    e = corr::launch_xeng_f32(a, sb, L.bt, aligned, q->stream);
  if (e != hipSuccess) return CORR_E_HIP;
  if (!direct) {
    e = corr::launch_reduce_splits(q->part, (int64_t)c.n_channels * L.n_products, split, q->acc, q->accumulate,
                                   is_int, q->stream);
    if (e != hipSuccess) return CORR_E_HIP;
  }
  return CORR_OK;
}

namespace {

// Integer-sample bounds: |Re V|, |Im V| <= 2 max_abs^2 n.
bool within(const corr_config& c, int64_t n, double limit) {
  return 2.0 * (double)c.max_abs * (double)c.max_abs * (double)n <= limit;
}

}  // namespace

extern "C" {

const char* corr_status_str(corr_status s) {
  switch (s) {
    case CORR_OK: return "ok";
    case CORR_E_INVAL: return "invalid argument";
    case CORR_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case CORR_E_HIP: return "HIP runtime error";
    case CORR_E_STATE: return "plan in error state or wrong call order";
    case CORR_E_OVERFLOW: return "accumulation would exceed the exactness/overflow bound";
    case CORR_E_SEQ: return "sample block sequence gap or duplicate";
    case CORR_E_BUSY: return "ring buffer full or result not ready";
    case CORR_E_UNSUPPORTED: return "unsupported configuration";
    case CORR_E_CORRUPT: return "a workspace guard band was overwritten";
  }
  return "unknown status";
}

corr_status corr_workspace_bytes(const corr_config* cfg, size_t* bytes) {
  try {
    if (!bytes) return CORR_E_INVAL;
    const corr_status v = validate(cfg);
    if (v != CORR_OK) return v;
    *bytes = layout_of(cfg).total;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_create(const corr_config* cfg, void* d_workspace, size_t ws_bytes, void* hip_stream,
                        corr_plan** out) {
  try {
    if (!out) return CORR_E_INVAL;
    const corr_status v = validate(cfg);
    if (v != CORR_OK) return v;
    const Layout L = layout_of(cfg);
    if (!d_workspace || ws_bytes < L.total || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0)
      return CORR_E_WORKSPACE;
    corr_plan* p = new (std::nothrow) corr_plan();
    if (!p) return CORR_E_INVAL;
    p->cfg = *cfg;
    p->L = L;
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->ws = static_cast<uint8_t*>(d_workspace);
    hipError_t e = hipSuccess;
    if (cfg->fp64_longrun) e = corr::launch_fill_zero(at(p, L.longrun), (int64_t)align_up(L.longrun_bytes, 16), p->stream);
    if (e == hipSuccess && cfg->fft_size != 0) {
      const int N = cfg->fft_size;
      p->tw_host.resize(N);
      for (int m = 0; m < N; ++m) {
        const double ang = 2.0 * M_PI * (double)m / (double)N;
        p->tw_host[m] = make_float2((float)std::cos(ang), (float)-std::sin(ang));
      }
      e = hipMemcpyAsync(at(p, L.tw), p->tw_host.data(), N * sizeof(float2), hipMemcpyHostToDevice, p->stream);
      if (e == hipSuccess && cfg->pfb_taps > 1) {
        // Prototype filter: Hamming window times sinc((m - (PN-1)/2)/N), in FP64, stored as float.
        const int64_t len = (int64_t)cfg->pfb_taps * N;
        p->pfb_host.resize(len);
        for (int64_t m = 0; m < len; ++m) {
          const double w = 0.54 - 0.46 * std::cos(2.0 * M_PI * (double)m / (double)(len - 1));
          const double x = ((double)m - 0.5 * (double)(len - 1)) / (double)N;
          const double sinc = (x == 0.0) ? 1.0 : std::sin(M_PI * x) / (M_PI * x);
          p->pfb_host[m] = (float)(w * sinc);
        }
        e = hipMemcpyAsync(at(p, L.pfb), p->pfb_host.data(), len * sizeof(float), hipMemcpyHostToDevice, p->stream);
      }
    }
    if (e != hipSuccess) {
      delete p;
      return CORR_E_HIP;
    }
    *out = p;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_destroy(corr_plan* plan) {
  delete plan;
  return CORR_OK;
}

corr_status corr_aggregate_w16(const uint16_t* d_records, int32_t n_streams, int32_t words_per_record,
                               int64_t n_records, uint32_t first_counter, uint16_t* d_out, uint32_t* d_bad_records,
                               void* hip_stream) {
  if (n_streams < 1 || words_per_record < 1 || n_records < 0) return CORR_E_INVAL;
  if (n_records > 0 && (!d_records || !d_out)) return CORR_E_INVAL;
  const hipError_t e = corr::launch_aggregate_w16(d_records, n_streams, words_per_record, n_records, first_counter,
                                                  d_out, d_bad_records, static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? CORR_OK : (e == hipErrorInvalidValue ? CORR_E_INVAL : CORR_E_HIP);
}

corr_status corr_cmac_design(int32_t design, int32_t group, const float* d_spectra, int64_t n_samples,
                             int32_t n_inputs, int32_t n_channels, float* d_out, int32_t accumulate,
                             void* hip_stream) {
  if (design != CORR_DESIGN_PP && design != CORR_DESIGN_GP && design != CORR_DESIGN_HG) return CORR_E_INVAL;
  if (design == CORR_DESIGN_PP ? group != 1 : (group != 2 && group != 4)) return CORR_E_INVAL;
  if (n_inputs < 1 || n_channels < 1 || n_samples < 0 || n_inputs % group != 0) return CORR_E_INVAL;
  if (!d_spectra || !d_out) return CORR_E_INVAL;
  if (n_inputs > 128) return CORR_E_UNSUPPORTED;
  const hipError_t e = corr::launch_cmac_design(design, group, reinterpret_cast<const float2*>(d_spectra), n_samples,
                                                n_inputs, n_channels, reinterpret_cast<float2*>(d_out), accumulate,
                                                static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? CORR_OK : (e == hipErrorInvalidValue ? CORR_E_INVAL : CORR_E_HIP);
}

corr_status corr_seq_reset(corr_plan* p) {
  if (!p) return CORR_E_INVAL;
  if (p->error) return CORR_E_STATE;
  p->seq_valid = false;
  return CORR_OK;
}

corr_status corr_state(const corr_plan* p, int64_t* n_long, uint64_t* next_seq, int32_t* seq_valid) {
  if (!p) return CORR_E_INVAL;
  if (n_long) *n_long = p->n_long;
  if (next_seq) *next_seq = p->next_seq;
  if (seq_valid) *seq_valid = p->seq_valid ? 1 : 0;
  return CORR_OK;
}

corr_status corr_restore(corr_plan* p, const void* longrun, int32_t src_is_device, int64_t n_long,
                         uint64_t next_seq, int32_t seq_valid) {
  try {
    if (!p) return CORR_E_INVAL;
    if (p->error) return CORR_E_STATE;
    if (!p->cfg.fp64_longrun || !longrun || n_long < 0) return CORR_E_INVAL;
    hipError_t e = ensure_guards(p);
    if (e == hipSuccess)
      e = hipMemcpyAsync(at(p, p->L.longrun), longrun, p->L.longrun_bytes,
                         src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e);
    p->n_long = n_long;
    p->next_seq = next_seq;
    p->seq_valid = seq_valid != 0;
    p->acc_zero = true;
    p->n_accum = 0;
    p->ring_fill = 0;
    p->stage_fill = 0;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_channelise(corr_plan* p, const void* d_volt, int64_t n_blocks, uint64_t first_seq,
                            float* d_spectra_dbg) {
  try {
    if (!p) return CORR_E_INVAL;
    if (p->error) return CORR_E_STATE;
    const corr_config& c = p->cfg;
    if (c.fft_size == 0) return CORR_E_STATE;
    if (n_blocks < 0 || (n_blocks > 0 && !d_volt)) return CORR_E_INVAL;
    if (p->seq_valid && first_seq != p->next_seq) return CORR_E_SEQ;
    if (p->ring_fill + n_blocks > c.ring_samples) return CORR_E_BUSY;
    if (n_blocks > 0) {
      const hipError_t eg = ensure_guards(p);
      if (eg != hipSuccess) return hip_fail(p, eg);
      corr::FStageCall fc;
      fc.volt = d_volt;
      fc.twiddle = static_cast<const float2*>(at(p, p->L.tw));
      fc.ring = static_cast<int8_t*>(at(p, p->L.ring));
      fc.dbg = d_spectra_dbg;
      fc.n_blocks = n_blocks;
      fc.ring_stride = p->L.ring_stride;
      fc.t_offset = p->ring_fill;
      fc.n_in = c.n_inputs;
      fc.scale = c.requant_scale;
      fc.max_abs = (float)c.max_abs;
      fc.format = c.volt_format;
      fc.pfb_taps = c.pfb_taps;
      fc.pfb = c.pfb_taps > 1 ? static_cast<const float*>(at(p, p->L.pfb)) : nullptr;
      const hipError_t e = (c.volt_format == CORR_VOLT_R8) ? corr::launch_fstage_call(fc, p->stream)
                                                          : corr::launch_fstage_complex(fc, p->stream);
      if (e != hipSuccess) return hip_fail(p, e);
    }
    p->ring_fill += n_blocks;
    p->seq_valid = true;
    p->next_seq = first_seq + (uint64_t)n_blocks;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_correlate(corr_plan* p, const void* d_samples, int64_t n_samples, int64_t row_stride) {
  try {
    if (!p) return CORR_E_INVAL;
    if (p->error) return CORR_E_STATE;
    const corr_config& c = p->cfg;
    const void* x;
    int sb;
    int64_t n, stride;
    if (d_samples == nullptr && c.fft_size == 0) {
      // No ring to drain: only an empty pass (n_samples == 0) is meaningful.
      return n_samples == 0 ? CORR_OK : CORR_E_INVAL;
    }
    if (d_samples == nullptr) {
      x = at(p, p->L.ring);
      sb = 2;
      n = p->ring_fill;
      stride = p->L.ring_stride;
    } else {
      if (n_samples < 0 || row_stride < 0) return CORR_E_INVAL;
      x = d_samples;
      sb = (c.sample_type == CORR_CI8) ? 2 : (c.sample_type == CORR_CI4 ? 1 : 8);
      n = n_samples;
      stride = row_stride == 0 ? n_samples : row_stride;
      if (stride < n) return CORR_E_INVAL;
      if ((reinterpret_cast<uintptr_t>(x) % (sb == 8 ? 4 : sb)) != 0) return CORR_E_INVAL;
      // CI4 rows are staged 16 bytes at a time
      if (c.sample_type == CORR_CI4 && n > 0 && ((reinterpret_cast<uintptr_t>(x) % 16) != 0 || stride % 16 != 0))
        return CORR_E_UNSUPPORTED;
    }
    const int64_t total = p->n_accum + n;
    if (c.max_abs > 0) {
      // CI4 sums run at 256 times the visibility inside the engine
      const double i32 = c.sample_type == CORR_CI4 ? 2147483647.0 / 256.0 : 2147483647.0;
      if (c.engine == CORR_X_I8 && !within(c, total, i32)) return CORR_E_OVERFLOW;
      if ((c.engine == CORR_X_FP32 || c.engine == CORR_X_FP32M) && !within(c, total, 16777216.0))
        return CORR_E_OVERFLOW;
    }
    if (n > 0) {
      const hipError_t eg = ensure_guards(p);
      if (eg != hipSuccess) return hip_fail(p, eg);
    }
    if ((c.engine == CORR_X_F16 || c.engine == CORR_X_F8) && c.ring_samples == 0) {
      // Convert while staging (one pass over the float32 samples; FP8 first
      // takes the per-channel maximum of this call's samples).
      if ((reinterpret_cast<uintptr_t>(x) % 8) != 0) return CORR_E_UNSUPPORTED;
      const bool f8 = c.engine == CORR_X_F8;
      if (f8 && n > 0) {
        const hipError_t e = corr::launch_absmax(static_cast<const float*>(x), c.n_channels, c.n_inputs, n, stride,
                                                 static_cast<uint32_t*>(at(p, p->L.mbits)), p->stream);
        if (e != hipSuccess) return hip_fail(p, e);
      }
      const corr_status st = xengine_pass(p, x, f8 ? 2 : 4, n, stride, f8 ? corr::kElemF8Cvt : corr::kElemF16Cvt,
                                          nullptr, f8 ? static_cast<const uint32_t*>(at(p, p->L.mbits)) : nullptr);
      if (st != CORR_OK) return st;
      p->n_accum = total;
      return CORR_OK;
    }
    if (c.engine == CORR_X_F16 || c.engine == CORR_X_F8) {
      // Stage chunks of at most ring_samples samples, then correlate each.
      const int elem = (c.engine == CORR_X_F16) ? corr::kElemF16 : corr::kElemF8;
      for (int64_t t0 = 0; t0 < n; t0 += c.ring_samples) {
        const int64_t nt = std::min<int64_t>(c.ring_samples, n - t0);
        corr::LowpCall lc;
        lc.x = static_cast<const float*>(x) + t0 * 2;
        lc.n_ch = c.n_channels;
        lc.n_in = c.n_inputs;
        lc.n_t = nt;
        lc.row_stride = stride;
        lc.out_stride = p->L.stage_stride;
        lc.elem = elem;
        lc.out = at(p, p->L.stage);
        lc.m_bits = static_cast<uint32_t*>(at(p, p->L.mbits));
        lc.inv_scale2 = static_cast<float*>(at(p, p->L.scales));
        const hipError_t e = corr::launch_lowp_stage(lc, p->stream);
        if (e != hipSuccess) return hip_fail(p, e);
        const corr_status st = xengine_pass(p, at(p, p->L.stage), p->L.stage_sb, nt, p->L.stage_stride, elem,
                                            elem == corr::kElemF8 ? lc.inv_scale2 : nullptr);
        if (st != CORR_OK) return st;
        p->stage_fill = nt;
      }
      p->n_accum = total;
      return CORR_OK;
    }
    const int elem = c.engine == CORR_X_FP32M ? corr::kElemF32 : (c.sample_type == CORR_CI4 && d_samples ? corr::kElemCI4 : -1);
    const corr_status s = xengine_pass(p, x, sb, n, stride, elem);
    if (s != CORR_OK) return s;
    p->n_accum = total;
    if (d_samples == nullptr) p->ring_fill = 0;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_ring_read(corr_plan* p, void* dst, int32_t dst_is_device, int64_t* n_samples_out) {
  try {
    if (!p || !dst) return CORR_E_INVAL;
    if (p->error) return CORR_E_STATE;
    const corr_config& c = p->cfg;
    if (c.fft_size == 0) return CORR_E_STATE;
    const int64_t n = p->ring_fill;
    const int64_t rows = (int64_t)c.n_channels * c.n_inputs;
    hipError_t e = hipSuccess;
    if (n > 0) {
      e = hipMemcpy2DAsync(dst, (size_t)n * 2, at(p, p->L.ring), (size_t)p->L.ring_stride * 2, (size_t)n * 2,
                           (size_t)rows, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           p->stream);
      if (e != hipSuccess) return hip_fail(p, e);
    }
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e);
    if (n_samples_out) *n_samples_out = n;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_stage_read(corr_plan* p, void* dst, float* scales, int64_t* n_samples_out) {
  try {
    if (!p || !dst) return CORR_E_INVAL;
    if (p->error) return CORR_E_STATE;
    const corr_config& c = p->cfg;
    if (c.engine != CORR_X_F16 && c.engine != CORR_X_F8) return CORR_E_STATE;
    if (c.ring_samples == 0) return CORR_E_STATE;   // converting plan: nothing staged
    const int64_t n = p->stage_fill;
    const int64_t rows = (int64_t)c.n_channels * c.n_inputs;
    const int sb = p->L.stage_sb;
    hipError_t e = hipSuccess;
    if (n > 0) {
      e = hipMemcpy2DAsync(dst, (size_t)n * sb, at(p, p->L.stage), (size_t)p->L.stage_stride * sb, (size_t)n * sb,
                           (size_t)rows, hipMemcpyDeviceToHost, p->stream);
      if (e != hipSuccess) return hip_fail(p, e);
    }
    std::vector<float> inv;
    if (scales && c.engine == CORR_X_F8) {
      inv.resize(c.n_channels);
      e = hipMemcpyAsync(inv.data(), at(p, p->L.scales), inv.size() * sizeof(float), hipMemcpyDeviceToHost,
                         p->stream);
      if (e != hipSuccess) return hip_fail(p, e);
    }
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e);
    if (scales) {
      for (int32_t k = 0; k < c.n_channels; ++k)
        scales[k] = (c.engine == CORR_X_F8) ? (float)(1.0 / std::sqrt((double)inv[k])) : 1.0f;
    }
    if (n_samples_out) *n_samples_out = n;
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

corr_status corr_internal_dump_async(corr_plan* p, void* dst, int32_t dst_is_device, int64_t* n_samples_out) {
  if (!p || !dst) return CORR_E_INVAL;
  if (p->error) return CORR_E_STATE;
  if (p->acc_zero) return CORR_E_STATE;  // nothing accumulated
  const hipError_t e = hipMemcpyAsync(dst, at(p, p->L.acc), p->L.acc_bytes,
                                      dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, p->stream);
  if (e != hipSuccess) return hip_fail(p, e);
  if (n_samples_out) *n_samples_out = p->n_accum;
  p->acc_zero = true;
  p->n_accum = 0;
  return CORR_OK;
}

corr_status corr_dump_bytes(const corr_plan* p, int32_t what, size_t* bytes) {
  if (!p || !bytes) return CORR_E_INVAL;
  if (what & CORR_DUMP_LONGRUN) {
    if (!p->cfg.fp64_longrun) return CORR_E_INVAL;
    *bytes = p->L.longrun_bytes;
  } else {
    *bytes = p->L.acc_bytes;
  }
  return CORR_OK;
}

corr_status corr_dump(corr_plan* p, int32_t what, void* dst, int32_t dst_is_device, int64_t* n_samples_out,
                      int32_t* exact_out) {
  try {
    if (!p) return CORR_E_INVAL;
    if (p->error) return CORR_E_STATE;
    const corr_config& c = p->cfg;
    const Layout& L = p->L;
    const bool integ = (what & CORR_DUMP_INTEG) != 0;
    const bool longrun = (what & CORR_DUMP_LONGRUN) != 0;
    const bool fold = (what & CORR_DUMP_FOLD) != 0;
    if (what & ~(CORR_DUMP_INTEG | CORR_DUMP_LONGRUN | CORR_DUMP_FOLD | CORR_DUMP_NO_RESET)) return CORR_E_INVAL;
    if (integ && longrun) return CORR_E_INVAL;
    if ((integ || longrun) && !dst) return CORR_E_INVAL;
    if ((longrun || fold) && !c.fp64_longrun) return CORR_E_INVAL;
    hipError_t e = hipSuccess;
    const bool is_int = (c.engine == CORR_X_I8);
    if (fold && !p->acc_zero) {
      e = corr::launch_fold_f64(static_cast<double*>(at(p, L.longrun)), at(p, L.acc),
                                (int64_t)c.n_channels * L.n_products * 2, is_int, p->stream);
      if (e != hipSuccess) return hip_fail(p, e);
      p->n_long += p->n_accum;
    }
    const hipMemcpyKind kind = dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (integ) {
      if (p->acc_zero) {
        if (dst_is_device) {
          e = (L.acc_bytes % 16 == 0 && (reinterpret_cast<uintptr_t>(dst) & 15) == 0)
                  ? corr::launch_fill_zero(dst, (int64_t)L.acc_bytes, p->stream)
                  : corr::launch_fill_zero_bytes(dst, (int64_t)L.acc_bytes, p->stream);
        }
      } else {
        e = hipMemcpyAsync(dst, at(p, L.acc), L.acc_bytes, kind, p->stream);
      }
      if (e != hipSuccess) return hip_fail(p, e);
    }
    if (longrun) {
      e = hipMemcpyAsync(dst, at(p, L.longrun), L.longrun_bytes, kind, p->stream);
      if (e != hipSuccess) return hip_fail(p, e);
    }
    // A plain reset (no copy, no fold) queues nothing and need not wait.
    // Dumps that wait also check the workspace's guard bands.
    uint32_t bad = 0;
    if (integ || longrun || fold) {
      if (p->guards_set) {
        uint32_t* word = static_cast<uint32_t*>(at(p, L.status));
        e = corr::launch_guard_check(p->ws, L.guards, word, p->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, word, sizeof(bad), hipMemcpyDeviceToHost, p->stream);
        if (e != hipSuccess) return hip_fail(p, e);
      }
      e = hipStreamSynchronize(p->stream);
      if (e != hipSuccess) return hip_fail(p, e);
      if (bad != 0) {
        p->error = true;
        return CORR_E_CORRUPT;
      }
    }
    if (integ && p->acc_zero && !dst_is_device) std::memset(dst, 0, L.acc_bytes);
    if (n_samples_out) *n_samples_out = p->n_accum;
    if (exact_out) {
      // Integer samples on the exact engines: every integration is exact
      // (corr_correlate refuses anything past the bound); the FP64 long-run
      // sum of exact integers stays exact while 2 max_abs^2 n_long <= 2^53.
      const bool exact_engine =
          (c.engine == CORR_X_I8 || c.engine == CORR_X_FP32 || c.engine == CORR_X_FP32M) && c.max_abs > 0;
      const bool long_exact = exact_engine && within(c, p->n_long, 9007199254740992.0);
      *exact_out = (integ && exact_engine) || (longrun && long_exact) ? 1 : 0;
    }
    if (!(what & CORR_DUMP_NO_RESET)) {
      p->acc_zero = true;
      p->n_accum = 0;
    }
    return CORR_OK;
  } catch (...) {
    return CORR_E_INVAL;
  }
}

}  // extern "C"
