// Plain FP32 X-engine: V_ij[c] += sum_t x_i[c,t] conj(x_j[c,t]) with FP32
// vector FMAs and FP32 accumulation, for complex float32 or complex int8
// samples (int8 converted exactly to float when staged).
//
// The cross-multiply-accumulate of Sec. 4 ("third step") on the vector ALUs,
// the precision the paper used throughout.  The paper's fastest design shares
// each input sample among a small group of products through shared memory
// (group parallel, G = 4).  Here a workgroup owns a BT x BT tile of the
// lower-triangle baseline matrix, stages KS samples of BT inputs per operand in
// LDS, and each thread keeps an (BT/16) x (BT/16) block of complex
// accumulators in registers, so every LDS read feeds BT/16 complex MACs.
// Integer-valued samples give exact sums while they stay below 2^24 (checked
// on the host).  Im of autos is written as exactly zero.
#include "common.h"
#include "launch.h"

namespace corr {

constexpr int kF32KS = 16;  // samples per LDS stage

template <typename T>
struct SampleTraits;
template <>
struct SampleTraits<float2> {
  static constexpr int kBytes = 8;
  static constexpr int kPerChunk = 2;   // samples per 16-byte global load
};
template <>
struct SampleTraits<int8_t> {
  static constexpr int kBytes = 2;
  static constexpr int kPerChunk = 8;
};

// Raw 16-byte chunk of samples t .. t+P-1 of one row.  ALIGNED (row stride
// and chunk start 16-byte aligned, so the chunk lies inside the row): one
// unconditional load from an address clamped into the valid region, so the
// compiler does not wait for it before the FMAs that follow; unpack() zeroes
// what lies outside.  Otherwise: sample by sample, zero outside.
template <typename S, bool ALIGNED>
__device__ __forceinline__ int4 load_raw(const int8_t* __restrict__ xc, int64_t row_stride_b, int row,
                                         int n_in, int64_t t, int64_t t1) {
  constexpr int P = SampleTraits<S>::kPerChunk;
  constexpr int B = SampleTraits<S>::kBytes;
  if (ALIGNED) {
    const int rc = row < n_in ? row : n_in - 1;
    const int64_t last = ((t1 - 1) / P) * P;
    const int64_t tc = t < last ? t : last;
    return *reinterpret_cast<const int4*>(xc + (int64_t)rc * row_stride_b + tc * B);
  } else {
    int w[4] = {0, 0, 0, 0};
    if (row < n_in) {
      const int8_t* p = xc + (int64_t)row * row_stride_b + t * B;
#pragma unroll
      for (int s = 0; s < P; ++s) {
        if (t + s < t1) {
          if constexpr (B == 8) {
            const int* f = reinterpret_cast<const int*>(p + 8 * s);
            w[2 * s] = f[0];
            w[2 * s + 1] = f[1];
          } else {
            const uint32_t h = *reinterpret_cast<const uint16_t*>(p + 2 * s);
            w[s >> 1] |= (int)(h << (16 * (s & 1)));
          }
        }
      }
    }
    return make_int4(w[0], w[1], w[2], w[3]);
  }
}

// Raw chunk -> P float2 samples (exact for int8), zero outside rows [0, n_in)
// and samples [.., t1).
template <typename S>
__device__ __forceinline__ void unpack(int4 raw, int row, int n_in, int64_t t, int64_t t1,
                                       float2 (&v)[SampleTraits<S>::kPerChunk]) {
  constexpr int P = SampleTraits<S>::kPerChunk;
  constexpr int B = SampleTraits<S>::kBytes;
  const int ws[4] = {raw.x, raw.y, raw.z, raw.w};
  if constexpr (B == 8) {
    v[0] = make_float2(__int_as_float(ws[0]), __int_as_float(ws[1]));
    v[1] = make_float2(__int_as_float(ws[2]), __int_as_float(ws[3]));
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[2 * q] = make_float2((float)(int8_t)(ws[q] & 0xFF), (float)(int8_t)((ws[q] >> 8) & 0xFF));
      v[2 * q + 1] = make_float2((float)(int8_t)((ws[q] >> 16) & 0xFF), (float)(int8_t)((ws[q] >> 24) & 0xFF));
    }
  }
  const bool row_ok = row < n_in;
#pragma unroll
  for (int s = 0; s < P; ++s)
    if (!row_ok || t + s >= t1) v[s] = make_float2(0.f, 0.f);
}

template <typename S, int BT, bool ALIGNED, bool DIAG>
__device__ __forceinline__ void xeng_f32_tile(const XArgs& a, float2 (*lds)[2][kF32KS][BT], int ch, int split,
                                              int I, int J) {
  constexpr int P = SampleTraits<S>::kPerChunk;
  constexpr int B = SampleTraits<S>::kBytes;
  constexpr int CPR = kF32KS / P;            // chunks per row per stage
  constexpr int CHUNKS = BT * CPR;           // per panel
  constexpr int LPT = (CHUNKS + 255) / 256;  // chunks per thread per panel
  constexpr int R = BT / 16;                 // rows (and cols) per thread
  constexpr int RH = R / 4;                  // groups of 4 rows per thread

  const int8_t* __restrict__ xc = static_cast<const int8_t*>(a.x) + (int64_t)ch * a.ch_stride_b;
  const int64_t n_t = a.k_bytes / B;
  const int64_t split_t = a.k_split_bytes / B;
  const int64_t t0 = (int64_t)split * split_t;
  const int64_t t1 = min(n_t, t0 + split_t);
  const int n_st = t1 > t0 ? (int)((t1 - t0 + kF32KS - 1) / kF32KS) : 0;

  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;

  int4 ga[LPT], gb[LPT];
  auto gload = [&](int st) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int c = tid + 256 * q;
      if (c < CHUNKS) {
        const int row = c % BT, kc = c / BT;
        const int64_t t = t0 + (int64_t)st * kF32KS + kc * P;
        ga[q] = load_raw<S, ALIGNED>(xc, a.row_stride_b, I * BT + row, a.n_in, t, t1);
        if (!DIAG) gb[q] = load_raw<S, ALIGNED>(xc, a.row_stride_b, J * BT + row, a.n_in, t, t1);
      }
    }
  };
  auto lstore = [&](int buf, int st) {
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
      const int c = tid + 256 * q;
      if (c < CHUNKS) {
        const int row = c % BT, kc = c / BT;
        const int64_t t = t0 + (int64_t)st * kF32KS + kc * P;
        float2 v[P];
        unpack<S>(ga[q], I * BT + row, a.n_in, t, t1, v);
#pragma unroll
        for (int s = 0; s < P; ++s) lds[buf][0][kc * P + s][row] = v[s];
        if (!DIAG) {
          unpack<S>(gb[q], J * BT + row, a.n_in, t, t1, v);
#pragma unroll
          for (int s = 0; s < P; ++s) lds[buf][1][kc * P + s][row] = v[s];
        }
      }
    }
  };

  float vr[R][R], vi[R][R];
#pragma unroll
  for (int m = 0; m < R; ++m)
#pragma unroll
    for (int n = 0; n < R; ++n) vr[m][n] = vi[m][n] = 0.f;

  if (n_st > 0) {
    gload(0);
    lstore(0, 0);
  }
  __syncthreads();
  for (int st = 0; st < n_st; ++st) {
    const int cur = st & 1;
    if (st + 1 < n_st) gload(st + 1);
    const float2 (*As)[BT] = lds[cur][0];
    const float2 (*Bs)[BT] = DIAG ? lds[cur][0] : lds[cur][1];
#pragma unroll 4
    for (int k = 0; k < kF32KS; ++k) {
      float2 av[R], bv[R];
#pragma unroll
      for (int h = 0; h < RH; ++h)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          av[4 * h + q] = As[k][ty * 4 + 64 * h + q];
          bv[4 * h + q] = Bs[k][tx * 4 + 64 * h + q];
        }
#pragma unroll
      for (int m = 0; m < R; ++m)
#pragma unroll
        for (int n = 0; n < R; ++n) {
          // (ar + i ai)(br - i bi): re = ar br + ai bi, im = ai br - ar bi
          vr[m][n] = fmaf(av[m].x, bv[n].x, vr[m][n]);
          vr[m][n] = fmaf(av[m].y, bv[n].y, vr[m][n]);
          vi[m][n] = fmaf(av[m].y, bv[n].x, vi[m][n]);
          vi[m][n] = fmaf(-av[m].x, bv[n].y, vi[m][n]);
        }
    }
    if (st + 1 < n_st) lstore(cur ^ 1, st + 1);
    __syncthreads();
  }

  float2* __restrict__ out = static_cast<float2*>(a.out) + (int64_t)split * a.out_split_stride +
                             (int64_t)ch * a.n_products;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int i = I * BT + ty * 4 + 64 * (m / 4) + (m % 4);
#pragma unroll
    for (int n = 0; n < R; ++n) {
      const int j = J * BT + tx * 4 + 64 * (n / 4) + (n % 4);
      if (i < a.n_in && j <= i) {
        float2* p = out + tri_index(i, j);
        const float re = vr[m][n];
        const float im = (i == j) ? 0.f : vi[m][n];
        if (a.accumulate) {
          float2 o = *p;
          o.x += re;
          o.y += im;
          *p = o;
        } else {
          *p = make_float2(re, im);
        }
      }
    }
  }
}

template <typename S, int BT, bool ALIGNED>
__global__ __launch_bounds__(256, 2) void xeng_f32_kernel(XArgs a) {
  __shared__ float2 lds[2][2][kF32KS][BT];
  const int64_t slot = blockIdx.x / kNumXcd;
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if (slot >= a.per_xcd || item >= a.n_items) return;
  const int tile = (int)(item % a.n_tiles);
  const int64_t rest = item / a.n_tiles;
  const int split = (int)(rest % a.n_split);
  const int ch = (int)(rest / a.n_split);
  int I, J;
  tile_decode(tile, I, J);
  if (I == J) xeng_f32_tile<S, BT, ALIGNED, true>(a, lds, ch, split, I, J);
  else xeng_f32_tile<S, BT, ALIGNED, false>(a, lds, ch, split, I, J);
}

template <typename S>
static hipError_t launch_f32_typed(const XArgs& a, int bt, bool aligned, hipStream_t s) {
  const int64_t grid = (int64_t)a.per_xcd * kNumXcd;
  if (bt == 128) {
    if (aligned) hipLaunchKernelGGL((xeng_f32_kernel<S, 128, true>), dim3((unsigned)grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((xeng_f32_kernel<S, 128, false>), dim3((unsigned)grid), dim3(256), 0, s, a);
  } else {
    if (aligned) hipLaunchKernelGGL((xeng_f32_kernel<S, 64, true>), dim3((unsigned)grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((xeng_f32_kernel<S, 64, false>), dim3((unsigned)grid), dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

// sample_bytes: 8 (complex float32) or 2 (complex int8).  bt: 64 or 128.
hipError_t launch_xeng_f32(const XArgs& a, int sample_bytes, int bt, bool aligned, hipStream_t s) {
  if ((int64_t)a.per_xcd * kNumXcd <= 0) return hipSuccess;
  if (sample_bytes == 8) return launch_f32_typed<float2>(a, bt, aligned, s);
  return launch_f32_typed<int8_t>(a, bt, aligned, s);
}

}  // namespace corr
