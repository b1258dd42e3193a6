// int8 MFMA X-engine: V_ij[c] += sum_t x_i[c,t] conj(x_j[c,t]) for complex
// int8 samples, int32 accumulation (exact within the host-checked bound).
//
// The cross-multiply-accumulate step of an FX correlator (Sec. 4, third step;
// Fig. 2's per-channel outer product) written as two real rank-k updates per
// channel.  With each input row stored as interleaved (re, im) bytes along
// K = 2T,
//     Re V = A B^T            (re_i re_j + im_i im_j summed over t)
//     Im V = A (iB)^T         (iB = (-im_j, re_j) pairs: im_i re_j - re_i im_j)
// so one staged B fragment feeds both products after a byte rotation done in
// registers.  The paper's designs reuse inputs across a small group of
// products through shared memory (group parallel, Sec. 4); here a workgroup
// owns a BT x BT tile of the baseline matrix, stages BT rows of each operand
// in LDS per K chunk, and every staged byte feeds BT products on the matrix
// cores (v_mfma_i32_32x32x32_i8).  Tiles cover the lower triangle only (the
// redundant half of Fig. 2 is never computed; inside diagonal tiles the
// strictly-upper wave blocks skip their MFMAs).
#include "common.h"
#include "launch.h"

namespace corr {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kI8KC = 128;            // K bytes per LDS stage (64 samples)
constexpr int kI8RS = kI8KC + 16;     // LDS row stride, padded: 8 consecutive
                                      // rows hit 8 distinct 16-byte bank groups

// (re0, im0, re1, im1) bytes -> (-im0, re0, -im1, re1): multiply two packed
// complex int8 samples by i.  |im| <= 127 so the negation never overflows.
__device__ __forceinline__ int rot_i(int w) {
  const uint32_t u = (uint32_t)w;
  const uint32_t im = (u >> 8) & 0x00FF00FFu;       // im bytes at positions 0, 2
  const uint32_t neg = 0x01000100u - im;            // per 16-bit lane: low byte = -im
  return (int)((neg & 0x00FF00FFu) | ((u << 8) & 0xFF00FF00u));
}

__device__ __forceinline__ v4i rot_i4(v4i v) {
  v4i r;
  r.x = rot_i(v.x);
  r.y = rot_i(v.y);
  r.z = rot_i(v.z);
  r.w = rot_i(v.w);
  return r;
}

// 16 bytes of row `row` starting at byte kk.
// Aligned form (row stride and kk multiples of 16): the load is unconditional,
// from an address clamped into the valid region, so the compiler never has to
// wait for it before the MFMAs that follow; the chunk is zeroed or tail-masked
// when it is stored to LDS (fix16).  Unaligned form (rows only 2-byte
// aligned): one complex sample at a time, zero outside the valid region.
template <bool ALIGNED>
__device__ __forceinline__ v4i load16(const int8_t* __restrict__ xc, int64_t row_stride_b, int row,
                                      int n_in, int64_t kk, int64_t k1) {
  if (ALIGNED) {
    const int rc = row < n_in ? row : n_in - 1;
    const int64_t last = ((k1 - 1) >> 4) << 4;
    const int64_t kc = kk < last ? kk : last;
    return *reinterpret_cast<const v4i*>(xc + (int64_t)rc * row_stride_b + kc);
  } else {
    v4i v = {0, 0, 0, 0};
    if (row >= n_in || kk >= k1) return v;
    const uint16_t* p16 = reinterpret_cast<const uint16_t*>(xc + (int64_t)row * row_stride_b + kk);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (kk + 2 * s < k1) w[s >> 1] |= (uint32_t)p16[s] << (16 * (s & 1));
    }
    v.x = (int)w[0];
    v.y = (int)w[1];
    v.z = (int)w[2];
    v.w = (int)w[3];
    return v;
  }
}

// Aligned form: zero a chunk outside rows [0, n_in) or past k1, and the bytes
// of a chunk that straddles k1 that lie at or past it.
__device__ __forceinline__ v4i fix16(v4i v, int row, int n_in, int64_t kk, int64_t k1) {
  if (row >= n_in || kk >= k1) return v4i{0, 0, 0, 0};
  const int64_t valid = k1 - kk;
  if (valid >= 16) return v;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int64_t lo = 4 * w;
    const int keep = valid >= lo + 4 ? 4 : (valid > lo ? (int)(valid - lo) : 0);
    const uint32_t m = keep >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keep)) - 1u);
    v[w] = (int)((uint32_t)v[w] & m);
  }
  return v;
}

// One baseline tile (I, J) of one channel over K bytes [k0, k1).  DIAG tiles
// (I == J) stage one panel that serves as both operands.
template <int BT, bool ALIGNED, bool DIAG>
__device__ __forceinline__ void xeng_i8_tile(const XArgs& a, int8_t (*lds)[2][BT * kI8RS], int ch,
                                             int split, int I, int J) {
  constexpr int WT = BT / 2;                 // wave tile (2 x 2 waves)
  constexpr int MB = WT / 32;                // 32 x 32 MFMA blocks per wave side
  constexpr int CPR = kI8KC / 16;            // 16-byte chunks per row per stage
  constexpr int LPT = BT * CPR / 256;        // chunks per thread per panel
  static_assert(LPT >= 1 && BT * CPR % 256 == 0, "tile/stage mismatch");

  const int8_t* __restrict__ xc = static_cast<const int8_t*>(a.x) + (int64_t)ch * a.ch_stride_b;
  const int64_t k0 = (int64_t)split * a.k_split_bytes;
  const int64_t k1 = min(a.k_bytes, k0 + a.k_split_bytes);
  const int n_kc = k1 > k0 ? (int)((k1 - k0 + kI8KC - 1) / kI8KC) : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool wave_idle = DIAG && (wm < wn);  // strictly upper block of a diagonal tile

  v4i ga[LPT], gb[LPT];
  auto gload = [&](int kc) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int c = tid + 256 * q;
      const int row = c / CPR, cc = c % CPR;
      const int64_t kk = k0 + (int64_t)kc * kI8KC + cc * 16;
      ga[q] = load16<ALIGNED>(xc, a.row_stride_b, I * BT + row, a.n_in, kk, k1);
      if (!DIAG) gb[q] = load16<ALIGNED>(xc, a.row_stride_b, J * BT + row, a.n_in, kk, k1);
    }
  };
  auto lstore = [&](int st, int kc) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int c = tid + 256 * q;
      const int row = c / CPR, cc = c % CPR;
      const int64_t kk = k0 + (int64_t)kc * kI8KC + cc * 16;
      v4i va = ga[q];
      if (ALIGNED) va = fix16(va, I * BT + row, a.n_in, kk, k1);
      *reinterpret_cast<v4i*>(&lds[st][0][row * kI8RS + cc * 16]) = va;
      if (!DIAG) {
        v4i vb = gb[q];
        if (ALIGNED) vb = fix16(vb, J * BT + row, a.n_in, kk, k1);
        *reinterpret_cast<v4i*>(&lds[st][1][row * kI8RS + cc * 16]) = vb;
      }
    }
  };

  v16i vr[MB][MB], vi[MB][MB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        vr[m][n][r] = 0;
        vi[m][n][r] = 0;
      }

  if (n_kc > 0) {
    gload(0);
    lstore(0, 0);
  }
  __syncthreads();

  const int frag_row = lane & 31;
  const int frag_k = (lane >> 5) * 16;
  for (int kc = 0; kc < n_kc; ++kc) {
    const int cur = kc & 1;
    if (kc + 1 < n_kc) gload(kc + 1);
    if (!wave_idle) {
      const int8_t* As = lds[cur][0];
      const int8_t* Bs = DIAG ? lds[cur][0] : lds[cur][1];
#pragma unroll
      for (int ks = 0; ks < kI8KC / 32; ++ks) {
        v4i af[MB], bf[MB], bj[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m)
          af[m] = *reinterpret_cast<const v4i*>(As + (wm * WT + m * 32 + frag_row) * kI8RS + ks * 32 + frag_k);
#pragma unroll
        for (int n = 0; n < MB; ++n) {
          bf[n] = *reinterpret_cast<const v4i*>(Bs + (wn * WT + n * 32 + frag_row) * kI8RS + ks * 32 + frag_k);
          bj[n] = rot_i4(bf[n]);
        }
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
          for (int n = 0; n < MB; ++n) {
            if (DIAG && wm == wn && m < n) continue;   // strictly upper 32x32 block
            vr[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[m], bf[n], vr[m][n], 0, 0, 0);
            vi[m][n] = __builtin_amdgcn_mfma_i32_32x32x32_i8(af[m], bj[n], vi[m][n], 0, 0, 0);
          }
      }
    }
    if (kc + 1 < n_kc) lstore(cur ^ 1, kc + 1);
    __syncthreads();
  }

  if (wave_idle) return;
  // Epilogue: 32x32 accumulator layout -- register r of lane l holds
  // row 8*(r/4) + 4*(l/32) + r%4, column l%32.
  int2* __restrict__ out = static_cast<int2*>(a.out) + (int64_t)split * a.out_split_stride +
                           (int64_t)ch * a.n_products;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n) {
      if (DIAG && wm == wn && m < n) continue;
      const int j = J * BT + wn * WT + n * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = I * BT + wm * WT + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i < a.n_in && j <= i) {
          int2* p = out + tri_index(i, j);
          const int re = vr[m][n][r];
          const int im = (i == j) ? 0 : vi[m][n][r];
          if (a.accumulate) {
            int2 o = *p;
            o.x += re;
            o.y += im;
            *p = o;
          } else {
            *p = make_int2(re, im);
          }
        }
      }
    }
}

template <int BT, bool ALIGNED>
__global__ __launch_bounds__(256, 2) void xeng_i8_kernel(XArgs a) {
  __shared__ __attribute__((aligned(16))) int8_t lds[2][2][BT * kI8RS];

  const int64_t slot = blockIdx.x / kNumXcd;
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if (slot >= a.per_xcd || item >= a.n_items) return;

  const int tile = (int)(item % a.n_tiles);
  const int64_t rest = item / a.n_tiles;
  const int split = (int)(rest % a.n_split);
  const int ch = (int)(rest / a.n_split);
  int I, J;
  tile_decode(tile, I, J);
  if (I == J) xeng_i8_tile<BT, ALIGNED, true>(a, lds, ch, split, I, J);
  else xeng_i8_tile<BT, ALIGNED, false>(a, lds, ch, split, I, J);
}

// Host-side launcher (called from corr.cpp).  bt is 64 or 128.
hipError_t launch_xeng_i8(const XArgs& a, int bt, bool aligned, hipStream_t s) {
  const int64_t grid = (int64_t)a.per_xcd * kNumXcd;
  if (grid <= 0) return hipSuccess;
  if (bt == 128) {
    if (aligned) hipLaunchKernelGGL((xeng_i8_kernel<128, true>), dim3((unsigned)grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((xeng_i8_kernel<128, false>), dim3((unsigned)grid), dim3(256), 0, s, a);
  } else {
    if (aligned) hipLaunchKernelGGL((xeng_i8_kernel<64, true>), dim3((unsigned)grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((xeng_i8_kernel<64, false>), dim3((unsigned)grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace corr
