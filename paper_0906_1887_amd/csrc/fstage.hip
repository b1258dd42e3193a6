// F-stage: real int8 voltages -> 256-point real DFT per (input, block) ->
// requantised complex int8 samples in the channel-major ring.
//
// Sec. 4, steps 1-2: the unpack reorders the time-major block (input index
// fastest) into per-input series and converts to float, then an FFT forms
// the spectra; for real samples 2 N_C points give N_C + 1 channels and the
// redundant half is ignored (Sec. 2, Sec. 4).  Here the unpack is fused into
// the load (the transpose happens in LDS), the two-for-one trick transforms
// two real inputs a, b at once as z = a + i b (X_a = (Z_k + conj Z_{N-k})/2,
// X_b = (Z_k - conj Z_{N-k})/(2i)), the 256-point complex FFT is a 16 x 16
// four-step transform (16 lanes per FFT, each doing radix-4 x radix-4 DFT16s in
// registers, one LDS exchange with inner twiddles), and the output is scaled,
// rounded half to even, clipped to +-max_abs and written as int8 (re, im) to
// ring[k][input][t] -- the channel-major corner turn the X-engine reads.
// Channels k = 0..127 are kept (DC kept, Nyquist dropped).
#include "common.h"
#include "launch.h"

namespace corr {

constexpr int kFN = 256;          // FFT length
constexpr int kFCh = kFN / 2;     // channels kept
constexpr int kFBlk = 16;         // blocks per workgroup
constexpr int kFIn = 8;           // inputs per workgroup (4 pairs)
constexpr int kFPairs = kFIn / 2;
constexpr int kFFtPerRound = 16;  // 256 threads / 16 lanes per FFT
constexpr int kFSRow = 17;        // padded row of the 16x16 exchange

struct FArgs {
  const int8_t* volt;      // [n_blocks*256][n_in]
  const float2* twiddle;   // W_256^m = exp(-2 pi i m / 256), m = 0..255
  int8_t* ring;            // [128][n_in][ring_stride][2]
  float* dbg;              // optional [128][n_in][n_blocks][2]
  int64_t n_blocks;
  int64_t ring_stride;     // samples per ring row
  int64_t t_offset;        // ring time index of block 0
  int32_t n_in;
  int32_t n_ig;            // input groups = ceil(n_in / 8)
  float scale;             // requantisation scale s
  float max_abs;
  int32_t vec_in;          // 1: n_in % 8 == 0 and volt 8-byte aligned
  int32_t vec_out;         // 1: t_offset % 8 == 0 and ring_stride % 8 == 0
  int64_t n_items;         // block groups x input groups
  int64_t per_xcd;         // ceil(n_items / 8)
};

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

__device__ __forceinline__ int8_t requant(float x, float s, float m) {
  float r = rintf(s * x);  // round half to even
  r = fminf(fmaxf(r, -m), m);
  return (int8_t)(int)r;
}

__global__ __launch_bounds__(256, 2) void fstage_kernel(FArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t vin[kFBlk * kFN][kFIn];            // 32 KB
  __shared__ __attribute__((aligned(16))) float2 S[kFFtPerRound][kFSRow * 16];       // 34 KB; slot f: lanes 16f..16f+15 only
  __shared__ __attribute__((aligned(16))) uint16_t O[kFCh][2][kFBlk];                // 8 KB
  __shared__ float2 tw[kFN];

  const int tid = threadIdx.x;
  // The n_ig workgroups of one block group read the same input rows; the
  // XCD remap puts them on one XCD (one L2), one after another.
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if ((int64_t)(blockIdx.x / kNumXcd) >= a.per_xcd || item >= a.n_items) return;
  const int ig = (int)(item % a.n_ig);
  const int64_t b0 = (item / a.n_ig) * kFBlk;
  const int i0 = ig * kFIn;

  tw[tid] = a.twiddle[tid];

  // Load [16 blocks * 256 samples][8 inputs] (zero outside): all 16 loads of
  // a thread are in flight before the first LDS write.
  constexpr int kLoads = kFBlk * kFN / 256;
  if (a.vec_in && b0 + kFBlk <= a.n_blocks) {
    uint2 w[kLoads];
    const int8_t* p = a.volt + (b0 * kFN + tid) * a.n_in + i0;
#pragma unroll
    for (int q = 0; q < kLoads; ++q) w[q] = *reinterpret_cast<const uint2*>(p + (int64_t)q * 256 * a.n_in);
#pragma unroll
    for (int q = 0; q < kLoads; ++q) *reinterpret_cast<uint2*>(&vin[tid + 256 * q][0]) = w[q];
  } else {
    for (int r = tid; r < kFBlk * kFN; r += 256) {
      const int64_t t = b0 * kFN + r;
      uint8_t bytes[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (t < a.n_blocks * kFN) {
        const int8_t* p = a.volt + t * a.n_in + i0;
#pragma unroll
        for (int q = 0; q < 8; ++q) bytes[q] = (i0 + q < a.n_in) ? (uint8_t)p[q] : 0u;
      }
      uint2 w;
      w.x = bytes[0] | (bytes[1] << 8) | (bytes[2] << 16) | ((uint32_t)bytes[3] << 24);
      w.y = bytes[4] | (bytes[5] << 8) | (bytes[6] << 16) | ((uint32_t)bytes[7] << 24);
      *reinterpret_cast<uint2*>(&vin[r][0]) = w;
    }
  }
  __syncthreads();

  // One round per input pair: FFT slot f transforms block f of the pair.
  const int f = tid >> 4;     // block of this FFT
  const int l = tid & 15;     // lane within the FFT
  const int64_t nb = min((int64_t)kFBlk, a.n_blocks - b0);
  float2 twl[16];             // this lane's inner twiddles W_256^(l k2), the same in every round
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) twl[k2] = tw[(l * k2) & (kFN - 1)];
  for (int pr = 0; pr < kFPairs; ++pr) {
    // Pass 1: lane n1 = l transforms z[n1 + 16 n2] over n2 (one 16-bit LDS
    // read gives both inputs of the pair).
    float2 x[16], X[16];
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) {
      const int r = f * kFN + l + 16 * n2;
      const uint32_t w = *reinterpret_cast<const uint16_t*>(&vin[r][2 * pr]);
      x[n2] = make_float2((float)(int8_t)(w & 0xFFu), (float)(int8_t)(w >> 8));
    }
    dft16(x, X);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) S[f][l * kFSRow + k2] = cmul(X[k2], twl[k2]);
    wave_sync();
    // Pass 2: lane k2 = l transforms over n1; output index k = k2 + 16 k1.
#pragma unroll
    for (int n1 = 0; n1 < 16; ++n1) x[n1] = S[f][n1 * kFSRow + l];
    dft16(x, X);
    wave_sync();
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) S[f][l + 16 * k1] = X[k1];
    wave_sync();
    // Split the two real inputs and requantise channels k < 128.
    const int64_t blk_g = b0 + f;
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1) {
      const int k = l + 16 * k1;
      const float2 zk = X[k1];
      const float2 zm = S[f][(kFN - k) & (kFN - 1)];
      const float2 xa = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      const float2 xb = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
      O[k][0][f] = (uint16_t)(uint8_t)requant(xa.x, a.scale, a.max_abs) |
                   ((uint16_t)(uint8_t)requant(xa.y, a.scale, a.max_abs) << 8);
      O[k][1][f] = (uint16_t)(uint8_t)requant(xb.x, a.scale, a.max_abs) |
                   ((uint16_t)(uint8_t)requant(xb.y, a.scale, a.max_abs) << 8);
      if (a.dbg != nullptr && blk_g < a.n_blocks) {
        const int ia = i0 + 2 * pr, ib = ia + 1;
        if (ia < a.n_in)
          reinterpret_cast<float2*>(a.dbg)[((int64_t)k * a.n_in + ia) * a.n_blocks + blk_g] = xa;
        if (ib < a.n_in)
          reinterpret_cast<float2*>(a.dbg)[((int64_t)k * a.n_in + ib) * a.n_blocks + blk_g] = xb;
      }
    }
    __syncthreads();
    // Write O[k][2 inputs][16 blocks] to ring[k][input][t_offset + b0 ..]:
    // one 32-byte row segment per thread.
    {
      const int k = tid >> 1, il = tid & 1;
      const int i = i0 + 2 * pr + il;
      if (i < a.n_in) {
        uint16_t* dst =
            reinterpret_cast<uint16_t*>(a.ring) + ((int64_t)k * a.n_in + i) * a.ring_stride + a.t_offset + b0;
        if (a.vec_out && nb == kFBlk) {
          const uint4* src = reinterpret_cast<const uint4*>(&O[k][il][0]);
          reinterpret_cast<uint4*>(dst)[0] = src[0];
          reinterpret_cast<uint4*>(dst)[1] = src[1];
        } else {
          for (int q = 0; q < nb; ++q) dst[q] = O[k][il][q];
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_fstage(const FArgs& a, hipStream_t s) {
  const int64_t n_bg = (a.n_blocks + kFBlk - 1) / kFBlk;
  FArgs b = a;
  b.n_items = n_bg * a.n_ig;
  if (b.n_items <= 0) return hipSuccess;
  b.per_xcd = (b.n_items + kNumXcd - 1) / kNumXcd;
  const int64_t grid = b.per_xcd * kNumXcd;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fstage_kernel, dim3((unsigned)grid), dim3(256), 0, s, b);
  return hipGetLastError();
}

}  // namespace corr

namespace corr {

hipError_t launch_fstage_call(const FStageCall& c, hipStream_t s) {
  FArgs a;
  a.volt = c.volt;
  a.twiddle = c.twiddle;
  a.ring = c.ring;
  a.dbg = c.dbg;
  a.n_blocks = c.n_blocks;
  a.ring_stride = c.ring_stride;
  a.t_offset = c.t_offset;
  a.n_in = c.n_in;
  a.n_ig = (c.n_in + kFIn - 1) / kFIn;
  a.scale = c.scale;
  a.max_abs = c.max_abs;
  a.vec_in = (c.n_in % kFIn == 0) && ((reinterpret_cast<uintptr_t>(c.volt) & 7) == 0);
  a.vec_out = (c.t_offset % 8 == 0) && (c.ring_stride % 8 == 0) && ((reinterpret_cast<uintptr_t>(c.ring) & 15) == 0);
  return launch_fstage(a, s);
}

}  // namespace corr
