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
// their bit patterns), one atomicMax per workgroup.
__global__ __launch_bounds__(256) void absmax_kernel(const float* __restrict__ x, int64_t n_in, int64_t n_t,
                                                      int64_t row_stride, int64_t rows_per_wg,
                                                      uint32_t* __restrict__ m_bits) {
  const int64_t ch = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t r1 = min(n_in, r0 + rows_per_wg);
  float m = 0.f;
  for (int64_t r = r0; r < r1; ++r) {
    const float* row = x + ((ch * n_in + r) * row_stride) * 2;
    for (int64_t k = threadIdx.x; k < 2 * n_t; k += blockDim.x) m = fmaxf(m, fabsf(row[k]));
  }
  __shared__ float red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(&m_bits[ch], __float_as_uint(red[0]));
}

// The exponent is clamped to [-60, 60] (so 1/s^2 stays a normal float) and
// the correction loops are bounded; within that range the result is exact,
// because s is a power of two and the comparisons are exact.
__device__ __forceinline__ float e4m3_scale(float m) {
  if (!(m > 0.f) || !(m < INFINITY)) return 1.f;
  const float e = fminf(fmaxf(floorf(log2f(448.f / m)), -60.f), 60.f);
  float s = ldexpf(1.f, (int)e);
  for (int k = 0; k < 4 && s * m > 448.f && s > 0x1p-60f; ++k) s *= 0.5f;
  for (int k = 0; k < 4 && 2.f * s * m <= 448.f && s < 0x1p60f; ++k) s *= 2.f;
  return s;
}

// One thread converts 4 complex samples of one row.  out rows have
// out_stride samples; elem 1: FP16 (4 bytes per sample), 2: FP8 (2 bytes).
template <int ELEM>
__global__ __launch_bounds__(256) void lowp_convert_kernel(const float* __restrict__ x, int64_t n_in, int64_t n_t,
                                                           int64_t row_stride, int64_t out_stride,
                                                           const uint32_t* __restrict__ m_bits, void* __restrict__ out,
                                                           float* __restrict__ inv_scale2) {
  const int64_t ch = blockIdx.y;
  const int64_t groups = (n_t + 3) / 4;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float s = 1.f;
  if (ELEM == kElemF8) {
    s = e4m3_scale(__uint_as_float(m_bits[ch]));
    if (gid == 0) inv_scale2[ch] = 1.f / (s * s);
  }
  if (gid >= n_in * groups) return;
  const int64_t r = gid / groups;
  const int64_t t0 = (gid - r * groups) * 4;
  const float* src = x + ((ch * n_in + r) * row_stride + t0) * 2;
  float v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = (t0 + q / 2 < n_t) ? src[q] : 0.f;
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

hipError_t launch_lowp_stage(const LowpCall& c, hipStream_t s) {
  if (c.n_ch <= 0 || c.n_in <= 0 || c.n_t <= 0) return hipSuccess;
  if (c.n_ch > 65535) return hipErrorInvalidValue;
  hipError_t e;
  if (c.elem == kElemF8) {
    e = launch_fill_zero(c.m_bits, (c.n_ch * 4 + 15) / 16 * 16, s);
    if (e != hipSuccess) return e;
    const int64_t rows_per_wg = 4;
    const dim3 g((unsigned)((c.n_in + rows_per_wg - 1) / rows_per_wg), (unsigned)c.n_ch);
    hipLaunchKernelGGL(absmax_kernel, g, dim3(256), 0, s, c.x, (int64_t)c.n_in, c.n_t, c.row_stride, rows_per_wg,
                       c.m_bits);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t groups = (c.n_t + 3) / 4;
  const dim3 g((unsigned)((c.n_in * groups + 255) / 256), (unsigned)c.n_ch);
  if (c.elem == kElemF16)
    hipLaunchKernelGGL(lowp_convert_kernel<kElemF16>, g, dim3(256), 0, s, c.x, (int64_t)c.n_in, c.n_t,
                       c.row_stride, c.out_stride, c.m_bits, c.out, c.inv_scale2);
  else
    hipLaunchKernelGGL(lowp_convert_kernel<kElemF8>, g, dim3(256), 0, s, c.x, (int64_t)c.n_in, c.n_t,
                       c.row_stride, c.out_stride, c.m_bits, c.out, c.inv_scale2);
  return hipGetLastError();
}

}  // namespace corr
