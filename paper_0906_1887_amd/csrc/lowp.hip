// Low-precision staging for the FP16 and FP8 X-engines: complex float32
// samples -> IEEE binary16 (unscaled) or OCP FP8 E4M3 with a per-channel
// power-of-two scale, both rounded to nearest even.
//
// FP8 scale: s_c = the largest power of two with s_c * m_c <= 448 (the largest
// finite E4M3 value), m_c = max |re|, |im| over the channel's inputs and
// samples in this chunk (s_c = 1 when m_c = 0 or not finite; s_c is kept in
// [2^-60, 2^60]).  Scaling by a power of two is
// exact in FP32, so the X-engine epilogue recovers V by multiplying by
// 1/s_c^2, also exactly.
#include "common.h"
#include "launch.h"

namespace corr {

// Max |re|, |im| per channel (as float bits; non-negative floats order like
// their bit patterns), one atomicMax per workgroup.  VEC: rows start 16-byte
// aligned, so each lane reads two complex samples (one float4) at a time.
template <bool VEC>
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ x, int64_t n_in, int64_t n_t,
                                                      int64_t row_stride, int64_t rows_per_wg,
                                                      uint32_t* __restrict__ m_bits) {
  const int64_t ch = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(n_in, r0 + rows_per_wg);
  const int tid = threadIdx.x;
  float m = 0.f;
  for (int64_t r = r0; r < r1; ++r) {
    const float* row = x + ((ch * n_in + r) * row_stride) * 2;
    if (VEC) {
      const float4* rv = reinterpret_cast<const float4*>(row);
      const int64_t nv = n_t / 2;
      int64_t u = tid;
      for (; u + 768 < nv; u += 1024) {
        const float4 a = rv[u], b = rv[u + 256], c = rv[u + 512], d = rv[u + 768];
        m = fmaxf(m, fmaxf(fmaxf(fmaxf(fabsf(a.x), fabsf(a.y)), fmaxf(fabsf(a.z), fabsf(a.w))),
                           fmaxf(fmaxf(fabsf(b.x), fabsf(b.y)), fmaxf(fabsf(b.z), fabsf(b.w)))));
        m = fmaxf(m, fmaxf(fmaxf(fmaxf(fabsf(c.x), fabsf(c.y)), fmaxf(fabsf(c.z), fabsf(c.w))),
                           fmaxf(fmaxf(fabsf(d.x), fabsf(d.y)), fmaxf(fabsf(d.z), fabsf(d.w)))));
      }
      for (; u < nv; u += 256) {
        const float4 a = rv[u];
        m = fmaxf(m, fmaxf(fmaxf(fabsf(a.x), fabsf(a.y)), fmaxf(fabsf(a.z), fabsf(a.w))));
      }
      if ((n_t & 1) && tid == 0) m = fmaxf(m, fmaxf(fabsf(row[2 * n_t - 2]), fabsf(row[2 * n_t - 1])));
    } else {
      for (int64_t k = tid; k < 2 * n_t; k += 256) m = fmaxf(m, fabsf(row[k]));
    }
  }
  __shared__ float red[256];
  red[tid] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] = fmaxf(red[tid], red[tid + w]);
    __syncthreads();
  }
  if (tid == 0) atomicMax(&m_bits[ch], __float_as_uint(red[0]));
}

// One thread converts 4 complex samples of one row (grid: sample groups x
// rows x channels).  Out rows have out_stride samples; FP16: 4 bytes per
// sample, FP8: 2.  VEC: the row starts 16-byte aligned, so full groups are
// read as two float4.
template <int ELEM, bool VEC>
__global__ __launch_bounds__(256) void lowp_convert_kernel(const float* __restrict__ x, int64_t n_in, int64_t n_t,
                                                           int64_t row_stride, int64_t out_stride,
                                                           const uint32_t* __restrict__ m_bits, void* __restrict__ out,
                                                           float* __restrict__ inv_scale2) {
  const int64_t ch = blockIdx.z;
  const int64_t r = blockIdx.y;
  const int64_t t0 = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  float s = 1.f;
  if (ELEM == kElemF8) {
    s = e4m3_scale(__uint_as_float(m_bits[ch]));
    if (r == 0 && t0 == 0) inv_scale2[ch] = 1.f / (s * s);
  }
  if (t0 >= n_t) return;
  const float* src = x + ((ch * n_in + r) * row_stride + t0) * 2;
  float v[8];
  if (VEC && t0 + 4 <= n_t) {
    const float4 a = reinterpret_cast<const float4*>(src)[0];
    const float4 b = reinterpret_cast<const float4*>(src)[1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (t0 + q / 2 < n_t) ? src[q] : 0.f;
  }
  if (ELEM == kElemF16) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // float -> _Float16 conversion rounds to nearest even (v_cvt_f16_f32)
      const uint32_t lo = __builtin_bit_cast(uint16_t, (_Float16)v[2 * q]);
      const uint32_t hi = __builtin_bit_cast(uint16_t, (_Float16)v[2 * q + 1]);
      w[q] = lo | (hi << 16);
    }
    uint32_t* dst = reinterpret_cast<uint32_t*>(out) + (ch * n_in + r) * out_stride + t0;
    if (t0 + 4 <= n_t) {
      *reinterpret_cast<uint4*>(dst) = make_uint4(w[0], w[1], w[2], w[3]);
    } else {
      for (int q = 0; q < 4 && t0 + q < n_t; ++q) dst[q] = w[q];
    }
  } else {
    int w0 = __builtin_amdgcn_cvt_pk_fp8_f32(s * v[0], s * v[1], 0, false);
    w0 = __builtin_amdgcn_cvt_pk_fp8_f32(s * v[2], s * v[3], w0, true);
    int w1 = __builtin_amdgcn_cvt_pk_fp8_f32(s * v[4], s * v[5], 0, false);
    w1 = __builtin_amdgcn_cvt_pk_fp8_f32(s * v[6], s * v[7], w1, true);
    uint16_t* dst = reinterpret_cast<uint16_t*>(out) + (ch * n_in + r) * out_stride + t0;
    if (t0 + 4 <= n_t) {
      *reinterpret_cast<uint2*>(dst) = make_uint2((uint32_t)w0, (uint32_t)w1);
    } else {
      const uint16_t h[4] = {(uint16_t)w0, (uint16_t)((uint32_t)w0 >> 16), (uint16_t)w1,
                             (uint16_t)((uint32_t)w1 >> 16)};
      for (int q = 0; q < 4 && t0 + q < n_t; ++q) dst[q] = h[q];
    }
  }
}

// Per-channel max |re|, |im| of complex float32 rows into m_bits (zeroed first).
hipError_t launch_absmax(const float* x, int64_t n_ch, int64_t n_in, int64_t n_t, int64_t row_stride, uint32_t* m_bits,
                         hipStream_t s) {
  if (n_ch <= 0 || n_in <= 0) return hipSuccess;
  if (n_ch > 65535) return hipErrorInvalidValue;
  hipError_t e = launch_fill_zero(m_bits, (n_ch * 4 + 15) / 16 * 16, s);
  if (e != hipSuccess || n_t <= 0) return e;
  const bool vec = (reinterpret_cast<uintptr_t>(x) % 16 == 0) && (row_stride % 2 == 0);
  const int64_t rows_per_wg = 4;
  const dim3 g((unsigned)((n_in + rows_per_wg - 1) / rows_per_wg), (unsigned)n_ch);
  if (vec)
    hipLaunchKernelGGL(absmax_kernel<true>, g, dim3(256), 0, s, x, n_in, n_t, row_stride, rows_per_wg, m_bits);
  else
    hipLaunchKernelGGL(absmax_kernel<false>, g, dim3(256), 0, s, x, n_in, n_t, row_stride, rows_per_wg, m_bits);
  return hipGetLastError();
}

hipError_t launch_lowp_stage(const LowpCall& c, hipStream_t s) {
  if (c.n_ch <= 0 || c.n_in <= 0 || c.n_t <= 0) return hipSuccess;
  if (c.n_ch > 65535 || c.n_in > 65535) return hipErrorInvalidValue;
  const bool vec = (reinterpret_cast<uintptr_t>(c.x) % 16 == 0) && (c.row_stride % 2 == 0);
  if (c.elem == kElemF8) {
    const hipError_t e = launch_absmax(c.x, c.n_ch, c.n_in, c.n_t, c.row_stride, c.m_bits, s);
    if (e != hipSuccess) return e;
  }
  const int64_t gx = ((c.n_t + 3) / 4 + 255) / 256;
  if (gx > 0x7FFFFFFF) return hipErrorInvalidValue;
  const dim3 g((unsigned)gx, (unsigned)c.n_in, (unsigned)c.n_ch);
#define CORR_CONVERT(EL, V)                                                                                   \
  hipLaunchKernelGGL((lowp_convert_kernel<EL, V>), g, dim3(256), 0, s, c.x, (int64_t)c.n_in, c.n_t, c.row_stride, \
                     c.out_stride, c.m_bits, c.out, c.inv_scale2)
  if (c.elem == kElemF16) {
    if (vec) CORR_CONVERT(kElemF16, true); else CORR_CONVERT(kElemF16, false);
  } else {
    if (vec) CORR_CONVERT(kElemF8, true); else CORR_CONVERT(kElemF8, false);
  }
#undef CORR_CONVERT
  return hipGetLastError();
}

}  // namespace corr
