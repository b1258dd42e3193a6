// Device helpers shared by the F-stage kernels: complex arithmetic, radix-4
// / radix-8 / radix-16 DFT building blocks, wave-local LDS ordering and the
// two-instruction requantiser.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace corr {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 w) {
  return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

// In-place forward 4-point DFT: (a, b, c, d) -> (X0, X1, X2, X3).
__device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d) {
  const float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = make_float2(t1.x + t3.y, t1.y - t3.x);   // t1 - i t3
  d = make_float2(t1.x - t3.y, t1.y + t3.x);   // t1 + i t3
}

// Forward 16-point DFT of x[0..15] into X[0..15] (X may alias nothing).
// n = n1 + 4 n2, k = k1 + 4 k2: inner DFT4 over n2, twiddle W16^(n1 k1),
// outer DFT4 over n1.
__device__ __forceinline__ void dft16(const float2 (&x)[16], float2 (&X)[16]) {
  const float c1 = 0.92387953251128675613f;   // cos(pi/8)
  const float s1 = 0.38268343236508977173f;   // sin(pi/8)
  const float h = 0.70710678118654752440f;    // sqrt(1/2)
  float2 A[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    float2 a = x[n1], b = x[n1 + 4], c = x[n1 + 8], d = x[n1 + 12];
    dft4(a, b, c, d);
    A[n1][0] = a;
    A[n1][1] = b;
    A[n1][2] = c;
    A[n1][3] = d;
  }
  // W16^m for m = n1*k1: 1 -> (c1,-s1), 2 -> (h,-h), 3 -> (s1,-c1),
  // 4 -> (0,-1), 6 -> (-h,-h), 9 -> (-c1, s1)
  A[1][1] = cmul(A[1][1], make_float2(c1, -s1));
  A[1][2] = cmul(A[1][2], make_float2(h, -h));
  A[1][3] = cmul(A[1][3], make_float2(s1, -c1));
  A[2][1] = cmul(A[2][1], make_float2(h, -h));
  A[2][2] = make_float2(A[2][2].y, -A[2][2].x);
  A[2][3] = cmul(A[2][3], make_float2(-h, -h));
  A[3][1] = cmul(A[3][1], make_float2(s1, -c1));
  A[3][2] = cmul(A[3][2], make_float2(-h, -h));
  A[3][3] = cmul(A[3][3], make_float2(-c1, s1));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a = A[0][k1], b = A[1][k1], c = A[2][k1], d = A[3][k1];
    dft4(a, b, c, d);
    X[k1] = a;
    X[k1 + 4] = b;
    X[k1 + 8] = c;
    X[k1 + 12] = d;
  }
}

// Orders the LDS accesses of one wave around an exchange among its own lanes:
// a wave's LDS instructions execute in program order, so only the compiler
// has to be kept from moving them (no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Requantisation q = clip(rne(h * v), +-m) in two instructions: adding
// 1.5 * 2^23 rounds h * v (exactly formed inside the FMA) to an integer with
// the FPU's round-half-to-even, and the clamp happens in that offset
// domain, where [M - m, M + m] is exact.  The low byte of the result's bit
// pattern is then q as a two's-complement int8 (the pattern is
// 0x4B400000 + q for |q| < 2^22; larger values are clamped first).
constexpr float kRqMagic = 12582912.0f;  // 1.5 * 2^23
__device__ __forceinline__ uint32_t requant_bits(float v, float h, float lo, float hi) {
  return __float_as_uint(__builtin_amdgcn_fmed3f(fmaf(v, h, kRqMagic), lo, hi));
}

// In-place forward 8-point DFT of x[0..7] into X[0..7]: two DFT4s over the
// even and odd samples, then X_k = E_k + W8^k O_k, X_{k+4} = E_k - W8^k O_k.
__device__ __forceinline__ void dft8(const float2 (&x)[8], float2 (&X)[8]) {
  const float h = 0.70710678118654752440f;  // sqrt(1/2)
  float2 e0 = x[0], e1 = x[2], e2 = x[4], e3 = x[6];
  float2 o0 = x[1], o1 = x[3], o2 = x[5], o3 = x[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // W8^1 = (h, -h), W8^2 = -i, W8^3 = (-h, -h)
  o1 = make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
  o2 = make_float2(o2.y, -o2.x);
  o3 = make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  X[0] = cadd(e0, o0);
  X[4] = csub(e0, o0);
  X[1] = cadd(e1, o1);
  X[5] = csub(e1, o1);
  X[2] = cadd(e2, o2);
  X[6] = csub(e2, o2);
  X[3] = cadd(e3, o3);
  X[7] = csub(e3, o3);
}

}  // namespace corr
