// Matrix-core X-engine for aligned sample rows: int8 (int32 accumulation),
// FP16 and OCP FP8 E4M3 (FP32 accumulation).
//
// V_ij[c] += sum_t x_i[c,t] conj(x_j[c,t]) -- the cross-multiply-accumulate
// of Sec. 4 (third step), per channel, over the lower-triangle baseline tiles
// of Fig. 2's outer product.  Each input row holds interleaved (re, im)
// elements along K = 2T, so per channel
//     Re V = A B^T            Im V = A (iB)^T,  iB = (-im_j, re_j)
// and iB is formed from the staged B fragment in registers (a byte or
// half-word rotation with a sign flip), so one LDS read feeds both products.
//
// Pipeline: a workgroup (4 waves, 2 x 2) owns a BT x BT tile of one channel.
// Operand rows are staged 64 K-bytes at a time straight from global memory
// into LDS (global_load_lds_dwordx4: no registers, no VALU), NS stages deep,
// so loads for stage s+NS-1 are in flight while stage s feeds the MFMAs; one
// barrier per stage.  LDS rows are 64 bytes with the four 16-byte chunks
// XOR-permuted by row so that the 32 rows of an MFMA fragment read hit
// distinct banks.  Rows past N_I are loaded from a clamped address and only
// ever reach outputs that are never stored; bytes past the valid K range are
// zeroed in LDS before use.  Tiles are numbered channel-major and remapped
// from blockIdx.x so that each XCD (and its L2) runs a contiguous range of
// channels.
#include <type_traits>

#include "common.h"
#include "launch.h"

namespace corr {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kMKC = 64;   // K bytes per stage
constexpr int kMNS = 4;    // pipeline stages

// 16-byte chunk c (0..3) of LDS row r lives at chunk c ^ swz(r).
__device__ __forceinline__ int swz(int r) { return (r >> 2) & 3; }

// Multiply packed complex elements by i: (re, im) -> (-im, re).
__device__ __forceinline__ int rot_i8(int w) {
  const uint32_t u = (uint32_t)w;
  const uint32_t im = (u >> 8) & 0x00FF00FFu;
  const uint32_t neg = 0x01000100u - im;            // low byte of each 16-bit lane = -im
  return (int)((neg & 0x00FF00FFu) | ((u << 8) & 0xFF00FF00u));
}
__device__ __forceinline__ int rot_f16(int w) {     // one complex half pair per dword
  const uint32_t u = (uint32_t)w;
  return (int)(((u >> 16) ^ 0x8000u) | (u << 16));
}
__device__ __forceinline__ int rot_f8(int w) {      // two complex fp8 pairs per dword
  const uint32_t u = (uint32_t)w;
  const uint32_t sw = ((u >> 8) & 0x00FF00FFu) | ((u << 8) & 0xFF00FF00u);
  return (int)(sw ^ 0x00800080u);
}

template <int EK>
__device__ __forceinline__ v4i rot4(v4i v) {
  v4i r;
  if constexpr (EK == kElemF32) {   // two complex float32 per 16 bytes: (re, im) -> (-im, re)
    r[0] = (int)((uint32_t)v[1] ^ 0x80000000u);
    r[1] = v[0];
    r[2] = (int)((uint32_t)v[3] ^ 0x80000000u);
    r[3] = v[2];
    return r;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    r[q] = EK == kElemI8 ? rot_i8(v[q]) : (EK == kElemF16 ? rot_f16(v[q]) : rot_f8(v[q]));
  return r;
}

template <int EK>
struct MAcc;
template <>
struct MAcc<kElemI8> { typedef v16i T; };
template <>
struct MAcc<kElemF16> { typedef v16f T; };
template <>
struct MAcc<kElemF8> { typedef v16f T; };

// One 64-byte K stage of a 32 x 32 block: fragments are two 16-byte reads per
// lane (K bytes g*16.. and 32+g*16.., g = lane / 32) of A and of B.
template <int EK>
__device__ __forceinline__ void mfma64(const v4i (&a)[2], const v4i (&b)[2], typename MAcc<EK>::T& acc) {
  if constexpr (EK == kElemI8) {
    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[0], b[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[1], b[1], acc, 0, 0, 0);
  } else if constexpr (EK == kElemF16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a[0]), __builtin_bit_cast(v8h, b[0]),
                                                  acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a[1]), __builtin_bit_cast(v8h, b[1]),
                                                  acc, 0, 0, 0);
  } else {
    const v8i a8 = {a[0][0], a[0][1], a[0][2], a[0][3], a[1][0], a[1][1], a[1][2], a[1][3]};
    const v8i b8 = {b[0][0], b[0][1], b[0][2], b[0][3], b[1][0], b[1][1], b[1][2], b[1][3]};
    // format 0 (FP8 E4M3) for both operands, unit E8M0 scales (127 = 2^0)
    acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc, 0, 0, 0, 127, 0, 127);
  }
}

template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

template <int EK, int BT, bool DIAG>
__device__ __forceinline__ void mfma_tile(const XArgs& a, int8_t* lds, int ch, int split, int I, int J) {
  constexpr int WT = BT / 2;                 // wave tile
  constexpr int MB = WT / 32;                // 32 x 32 blocks per wave side
  constexpr int PANEL = BT * kMKC;           // bytes per operand per stage
  constexpr int STAGE = PANEL * (DIAG ? 1 : 2);
  constexpr int QPW = BT / 16 / 4;           // 1 KB load instructions per operand per wave
  constexpr int LPW = QPW * (DIAG ? 1 : 2);  // load instructions per wave per stage
  using Acc = typename MAcc<EK>::T;

  const int8_t* __restrict__ xc = static_cast<const int8_t*>(a.x) + (int64_t)ch * a.ch_stride_b;
  const int64_t k0 = (int64_t)split * a.k_split_bytes;
  const int64_t k1 = min(a.k_bytes, k0 + a.k_split_bytes);
  const int n_st = k1 > k0 ? (int)((k1 - k0 + kMKC - 1) / kMKC) : 0;
  const int64_t last = ((k1 - 1) >> 4) << 4;  // last valid 16-byte chunk start

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool wave_idle = DIAG && (wm < wn);

  // This lane's part of each load instruction: LDS row lrow (of 16), chunk p.
  const int lrow = lane >> 2, p = lane & 3;
  const int8_t* gA[QPW];
  const int8_t* gB[QPW];
  int rowq[QPW];
#pragma unroll
  for (int q = 0; q < QPW; ++q) {
    const int r = (wave * QPW + q) * 16 + lrow;    // tile row
    rowq[q] = r;
    const int c = p ^ swz(r);                      // global chunk this lane fetches
    const int ra = min(I * BT + r, a.n_in - 1);
    gA[q] = xc + (int64_t)ra * a.row_stride_b + 16 * c;
    if (!DIAG) {
      const int rb = min(J * BT + r, a.n_in - 1);
      gB[q] = xc + (int64_t)rb * a.row_stride_b + 16 * c;
    }
  }

  auto issue = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE;
    const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
    for (int q = 0; q < QPW; ++q) {
      const int c = p ^ swz(rowq[q]);
      const int64_t kk = kb + 16 * c;
      const int64_t off = (kk <= last ? kb : last - 16 * c);   // keep the 16 bytes inside the row
      int8_t* dst = base + (wave * QPW + q) * 1024;
      __builtin_amdgcn_global_load_lds(gA[q] + off, dst, 16, 0, 0);
      if (!DIAG) __builtin_amdgcn_global_load_lds(gB[q] + off, dst + PANEL, 16, 0, 0);
    }
  };
  // Zero / mask the chunks of stage st that reach past k1 (only the last stage).
  auto fix_tail = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE;
    const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
    for (int q = 0; q < QPW; ++q) {
      const int c = p ^ swz(rowq[q]);
      const int64_t kk = kb + 16 * c;
      if (kk + 16 > k1) {
        const int64_t valid = k1 - kk;
#pragma unroll
        for (int op = 0; op < (DIAG ? 1 : 2); ++op) {
          v4i* cell = reinterpret_cast<v4i*>(base + op * PANEL + (wave * QPW + q) * 1024 + lane * 16);
          v4i v = *cell;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t lo = 4 * w;
            const int keep = valid >= lo + 4 ? 4 : (valid > lo ? (int)(valid - lo) : 0);
            const uint32_t m = keep >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keep)) - 1u);
            v[w] = (int)((uint32_t)v[w] & m);
          }
          *cell = v;
        }
      }
    }
  };

  Acc vr[MB][MB], vi[MB][MB];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int n = 0; n < MB; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        vr[m][n][r] = 0;
        vi[m][n][r] = 0;
      }

#pragma unroll
  for (int s = 0; s < kMNS - 1; ++s)
    if (s < n_st) issue(s);

  const int frow = lane & 31;
  const int g = lane >> 5;
  const bool tail = (k1 - k0) % kMKC != 0;
  for (int s = 0; s < n_st; ++s) {
    // Wait for this wave's loads of stage s; later stages may stay in flight.
    const int ahead = min(kMNS - 2, n_st - 1 - s);
    if (ahead >= 2) wait_vmcnt<2 * LPW>();
    else if (ahead == 1) wait_vmcnt<LPW>();
    else wait_vmcnt<0>();
    if (tail && s == n_st - 1) {
      fix_tail(s);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
    // Plain s_barrier (as asm with a memory clobber, so the compiler keeps
    // LDS reads below it): each wave has already waited for its own stage-s
    // loads, which is all the other waves need; a fenced barrier would also
    // drain the loads of later stages that are meant to stay in flight.
    asm volatile("s_barrier" ::: "memory");
    if (s + kMNS - 1 < n_st) issue(s + kMNS - 1);
    if (!wave_idle) {
      const int8_t* As = lds + (s % kMNS) * STAGE;
      const int8_t* Bs = DIAG ? As : As + PANEL;
      v4i af[MB][2], bf[MB][2], bj[MB][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int cidx = 2 * h + g;            // logical 16-byte chunk
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          const int r = wm * WT + m * 32 + frow;
          af[m][h] = *reinterpret_cast<const v4i*>(As + r * kMKC + 16 * (cidx ^ swz(r)));
        }
#pragma unroll
        for (int n = 0; n < MB; ++n) {
          const int r = wn * WT + n * 32 + frow;
          bf[n][h] = *reinterpret_cast<const v4i*>(Bs + r * kMKC + 16 * (cidx ^ swz(r)));
          bj[n][h] = rot4<EK>(bf[n][h]);
        }
      }
#pragma unroll
      for (int m = 0; m < MB; ++m)
#pragma unroll
        for (int n = 0; n < MB; ++n) {
          if (DIAG && wm == wn && m < n) continue;   // strictly upper 32 x 32 block
          mfma64<EK>(af[m], bf[n], vr[m][n]);
          mfma64<EK>(af[m], bj[n], vi[m][n]);
        }
    }
  }

  if (wave_idle) return;
  // Epilogue.  32 x 32 accumulator layout: register r of lane l holds row
  // 8*(r/4) + 4*(l/32) + r%4, column l%32.
  float scale = 1.0f;
  if constexpr (EK == kElemF8) scale = a.inv_scale2 ? a.inv_scale2[ch] : 1.0f;
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
          const int64_t off = (int64_t)split * a.out_split_stride + (int64_t)ch * a.n_products + tri_index(i, j);
          if constexpr (EK == kElemI8) {
            int2* pp = static_cast<int2*>(a.out) + off;
            const int re = vr[m][n][r];
            const int im = (i == j) ? 0 : vi[m][n][r];
            if (a.accumulate) {
              int2 o = *pp;
              o.x += re;
              o.y += im;
              *pp = o;
            } else {
              *pp = make_int2(re, im);
            }
          } else {
            float2* pp = static_cast<float2*>(a.out) + off;
            const float re = vr[m][n][r] * scale;
            const float im = (i == j) ? 0.f : vi[m][n][r] * scale;
            if (a.accumulate) {
              float2 o = *pp;
              o.x += re;
              o.y += im;
              *pp = o;
            } else {
              *pp = make_float2(re, im);
            }
          }
        }
      }
    }
}

// Multiply packed complex elements by -i: (re, im) -> (im, -re).
__device__ __forceinline__ int rotm_i8(int w) {
  const uint32_t u = (uint32_t)w;
  const uint32_t neg = 0x01000100u - (u & 0x00FF00FFu);   // low byte of each 16-bit lane = -re
  // bytes: im0 (u.1), -re0 (neg.0), im1 (u.3), -re1 (neg.2)
  return (int)__builtin_amdgcn_perm(neg, u, 0x06030401u);
}
__device__ __forceinline__ int rotm_f16(int w) {
  const uint32_t u = (uint32_t)w;
  return (int)(((u >> 16) | (u << 16)) ^ 0x80000000u);
}
__device__ __forceinline__ int rotm_f8(int w) {
  const uint32_t u = (uint32_t)w;
  const uint32_t sw = ((u >> 8) & 0x00FF00FFu) | ((u << 8) & 0xFF00FF00u);
  return (int)(sw ^ 0x80008000u);
}

template <int EK>
__device__ __forceinline__ v4i rotm4(v4i v) {
  v4i r;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    r[q] = EK == kElemI8 ? rotm_i8(v[q]) : (EK == kElemF16 ? rotm_f16(v[q]) : rotm_f8(v[q]));
  return r;
}

// One 32 x 32 block product over 16 K bytes per lane (int8: K = 32, FP16:
// K = 16).  FP8 blocks take both 16-byte halves at once (mfma64).
template <int EK>
__device__ __forceinline__ void mfma16(const v4i& a, const v4i& b, typename MAcc<EK>::T& acc) {
  static_assert(EK != kElemF8, "FP8 products span 32 K bytes per lane");
  if constexpr (EK == kElemI8) {
    acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a), __builtin_bit_cast(v8h, b), acc, 0, 0, 0);
  }
}

// 128 x 128 tile, four waves (2 x 2) of 64 x 64, two workgroups per CU so
// that each SIMD holds two waves.  Per stage a wave reads 8 fragments (A and
// B, two 32-row blocks each, two K halves) and issues 16 MFMAs (8 for FP8).
// Fragments are double-buffered in registers: the LDS reads of stage s+1 are
// interleaved with the MFMAs of stage s.  The barrier of stage s+1 follows
// every wave's completed reads of stage s, so stage s+NS may then be loaded
// into stage s's buffer.  Loads of stages that lie wholly inside the K range
// use uniform tile bases and 32-bit per-lane offsets (LDS destinations in
// scalar registers); the last stage clamps its addresses and is masked.
template <int EK, bool DIAG>
__device__ __forceinline__ void mfma_tile_128(const XArgs& a, int8_t* lds, int ch, int split, int I, int J) {
  constexpr int BT = 128;
  constexpr int PANEL = BT * kMKC;           // bytes per operand per stage
  constexpr int STAGE = PANEL * (DIAG ? 1 : 2);
  constexpr int QPW = BT / 16 / 4;           // 1 KB load instructions per operand per wave
  constexpr int LPW = QPW * (DIAG ? 1 : 2);  // load instructions per wave per stage
  constexpr int NMF = EK == kElemF8 ? 8 : 16;  // MFMAs per wave per stage
  using Acc = typename MAcc<EK>::T;

  const int8_t* __restrict__ xc = static_cast<const int8_t*>(a.x) + (int64_t)ch * a.ch_stride_b;
  const int64_t k0 = (int64_t)split * a.k_split_bytes;
  const int64_t k1 = min(a.k_bytes, k0 + a.k_split_bytes);
  const int n_st = k1 > k0 ? (int)((k1 - k0 + kMKC - 1) / kMKC) : 0;
  const int64_t last = ((k1 - 1) >> 4) << 4;   // last valid 16-byte chunk start
  // Stages whose 64 bytes all lie in [k0, k1) and whose offsets fit 32 bits.
  const int n_fast = a.row_stride_b < (int64_t(1) << 24) ? (int)((k1 - k0) / kMKC) : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  // This lane's part of each load instruction: LDS row lrow (of 16), chunk p.
  const int lrow = lane >> 2, p = lane & 3;
  const int8_t* gA[QPW];
  const int8_t* gB[QPW];
  uint32_t oA[QPW], oB[QPW];
  int rowq[QPW];
  const int8_t* tA = xc + (int64_t)(I * BT) * a.row_stride_b + k0;
  const int8_t* tB = xc + (int64_t)(J * BT) * a.row_stride_b + k0;
#pragma unroll
  for (int q = 0; q < QPW; ++q) {
    const int r = (wave * QPW + q) * 16 + lrow;    // tile row
    rowq[q] = r;
    const int c = p ^ swz(r);                      // global chunk this lane fetches
    const int ra = min(I * BT + r, a.n_in - 1);
    const int rb = min(J * BT + r, a.n_in - 1);
    gA[q] = xc + (int64_t)ra * a.row_stride_b + 16 * c;
    gB[q] = xc + (int64_t)rb * a.row_stride_b + 16 * c;
    oA[q] = (uint32_t)((int64_t)(ra - I * BT) * a.row_stride_b + 16 * c);
    oB[q] = (uint32_t)((int64_t)(rb - J * BT) * a.row_stride_b + 16 * c);
  }
  auto issue = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE + wave * QPW * 1024;
    if (st < n_fast) {
      const int8_t* ga = tA + st * kMKC;
      const int8_t* gb = tB + st * kMKC;
#pragma unroll
      for (int q = 0; q < QPW; ++q) {
        __builtin_amdgcn_global_load_lds(ga + oA[q], base + q * 1024, 16, 0, 0);
        if (!DIAG) __builtin_amdgcn_global_load_lds(gb + oB[q], base + q * 1024 + PANEL, 16, 0, 0);
      }
    } else {
      const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
      for (int q = 0; q < QPW; ++q) {
        const int c = p ^ swz(rowq[q]);
        const int64_t kk = kb + 16 * c;
        const int64_t off = (kk <= last ? kb : last - 16 * c);   // keep the 16 bytes inside the row
        __builtin_amdgcn_global_load_lds(gA[q] + off, base + q * 1024, 16, 0, 0);
        if (!DIAG) __builtin_amdgcn_global_load_lds(gB[q] + off, base + q * 1024 + PANEL, 16, 0, 0);
      }
    }
  };
  // Zero / mask the chunks of stage st that reach past k1 (only the last stage).
  auto fix_tail = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE;
    const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
    for (int q = 0; q < QPW; ++q) {
      const int c = p ^ swz(rowq[q]);
      const int64_t kk = kb + 16 * c;
      if (kk + 16 > k1) {
        const int64_t valid = k1 - kk;
#pragma unroll
        for (int op = 0; op < (DIAG ? 1 : 2); ++op) {
          v4i* cell = reinterpret_cast<v4i*>(base + op * PANEL + (wave * QPW + q) * 1024 + lane * 16);
          v4i v = *cell;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t lo = 4 * w;
            const int keep = valid >= lo + 4 ? 4 : (valid > lo ? (int)(valid - lo) : 0);
            const uint32_t m = keep >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keep)) - 1u);
            v[w] = (int)((uint32_t)v[w] & m);
          }
          *cell = v;
        }
      }
    }
  };

  Acc vr[2][2], vi[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        vr[m][n][r] = 0;
        vi[m][n][r] = 0;
      }

#pragma unroll
  for (int s = 0; s < kMNS - 1; ++s)
    if (s < n_st) issue(s);

  const int frow = lane & 31;
  const int g = lane >> 5;
  const bool tail = (k1 - k0) % kMKC != 0;
  // Wait for this wave's loads of stage st (later stages stay in flight),
  // mask the K tail, and make stage st visible to all waves.  A plain
  // s_barrier: a fenced one would also drain the later stages' loads.
  auto arrive = [&](int st) {
    const int ahead = min(kMNS - 2, n_st - 1 - st);
    if (ahead >= 2) wait_vmcnt<2 * LPW>();
    else if (ahead == 1) wait_vmcnt<LPW>();
    else wait_vmcnt<0>();
    if (tail && st == n_st - 1) fix_tail(st);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    asm volatile("s_barrier" ::: "memory");
  };
  auto read = [&](int st, v4i (&af)[2][2], v4i (&bf)[2][2]) {
    const int8_t* As = lds + (st % kMNS) * STAGE;
    const int8_t* Bs = DIAG ? As : As + PANEL;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cidx = 2 * h + g;              // logical 16-byte chunk
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int r = wm * 64 + m * 32 + frow;
        af[m][h] = *reinterpret_cast<const v4i*>(As + r * kMKC + 16 * (cidx ^ swz(r)));
      }
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const int r = wn * 64 + n * 32 + frow;
        bf[n][h] = *reinterpret_cast<const v4i*>(Bs + r * kMKC + 16 * (cidx ^ swz(r)));
      }
    }
  };
  // Re products first; the -i rotation of A runs on the VALU while they
  // execute, then the Im products: Im V = (-iA) B^T.  Consecutive MFMAs go to
  // different accumulators.  SK: a diagonal wave of a diagonal tile skips its
  // strictly upper block (m 0, n 1).
  auto compute = [&](auto sk, const v4i (&af)[2][2], const v4i (&bf)[2][2]) {
    constexpr bool SK = decltype(sk)::value;
    v4i ra[2][2];
    if constexpr (EK == kElemF8) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
          if (!(SK && m == 0 && n == 1)) mfma64<EK>(af[m], bf[n], vr[m][n]);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) ra[m][h] = rotm4<EK>(af[m][h]);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n)
          if (!(SK && m == 0 && n == 1)) mfma64<EK>(ra[m], bf[n], vi[m][n]);
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n)
            if (!(SK && m == 0 && n == 1)) mfma16<EK>(af[m][h], bf[n][h], vr[m][n]);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) ra[m][h] = rotm4<EK>(af[m][h]);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < 2; ++n)
            if (!(SK && m == 0 && n == 1)) mfma16<EK>(ra[m][h], bf[n][h], vi[m][n]);
    }
  };

  if (n_st > 0) {
    arrive(0);
    if (kMNS - 1 < n_st) issue(kMNS - 1);
  }
  // In a diagonal tile the wave of the strictly upper 64 x 64 quarter only
  // loads its share of the panel and keeps the barriers.
  if (DIAG && wm < wn) {
    for (int s = 0; s + 1 < n_st; ++s) {
      arrive(s + 1);
      if (s + kMNS < n_st) issue(s + kMNS);
    }
    return;
  }
  auto run = [&](auto sk) {
    constexpr int NM = (DIAG && decltype(sk)::value) ? NMF * 3 / 4 : NMF;   // MFMAs per stage
    v4i af0[2][2], bf0[2][2], af1[2][2], bf1[2][2];
    if (n_st > 0) read(0, af0, bf0);
    for (int s = 0; s + 1 < n_st; ++s) {
      arrive(s + 1);
      if (s + kMNS < n_st) issue(s + kMNS);
      read(s + 1, af1, bf1);
      compute(sk, af0, bf0);
#pragma unroll
      for (int q = 0; q < (NM < 8 ? NM : 8); ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      }
      if constexpr (NM > 8) __builtin_amdgcn_sched_group_barrier(0x008, NM - 8, 0);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          af0[m][h] = af1[m][h];
          bf0[m][h] = bf1[m][h];
        }
    }
    if (n_st > 0) compute(sk, af0, bf0);
  };
  if (DIAG && wm == wn) run(std::true_type{});
  else run(std::false_type{});

  // Epilogue.  32 x 32 accumulator layout: register r of lane l holds row
  // 8*(r/4) + 4*(l/32) + r%4, column l%32.
  float scale = 1.0f;
  if constexpr (EK == kElemF8) scale = a.inv_scale2 ? a.inv_scale2[ch] : 1.0f;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int j = J * BT + wn * 64 + n * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = I * BT + wm * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i < a.n_in && j <= i) {
          const int64_t off = (int64_t)split * a.out_split_stride + (int64_t)ch * a.n_products + tri_index(i, j);
          if constexpr (EK == kElemI8) {
            int2* pp = static_cast<int2*>(a.out) + off;
            const int re = vr[m][n][r];
            const int im = (i == j) ? 0 : vi[m][n][r];
            if (a.accumulate) {
              int2 o = *pp;
              o.x += re;
              o.y += im;
              *pp = o;
            } else {
              *pp = make_int2(re, im);
            }
          } else {
            float2* pp = static_cast<float2*>(a.out) + off;
            const float re = vr[m][n][r] * scale;
            const float im = (i == j) ? 0.f : vi[m][n][r] * scale;
            if (a.accumulate) {
              float2 o = *pp;
              o.x += re;
              o.y += im;
              *pp = o;
            } else {
              *pp = make_float2(re, im);
            }
          }
        }
      }
    }
}

// FP16 / FP8 engine reading complex float32 directly (plans without a
// staging chunk): the conversion of the staged engines moves into the load.
// A stage's float32 samples (FP16: 16 per row, 128 bytes; FP8: 32 per row,
// 256 bytes) are fetched with coalesced 16-byte loads (consecutive lanes read
// consecutive bytes of a row) into registers, PF stages ahead; each 16-byte
// load (two complex samples) is converted in registers (round to nearest
// even; FP8 after scaling by the channel's power of two s_c, saturating) and
// written to LDS in the staged engine's swizzled layout (8 bytes for FP16, 4
// for FP8).  The MFMA stage is that of mfma_tile_128, so the sums are those
// of the staged engine on the same codes.  Two LDS stage buffers, one
// barrier per stage, one workgroup per CU (the register prefetch takes the
// room of a second; cvt_waves below sets its wave count).  Samples past the
// pass are zero; rows past N_I are read from a clamped row and never stored.
constexpr int kPF = 3;   // stages of float32 samples in flight per workgroup (FP8; FP16 takes 4)

// Two floats -> two binary16 (round to nearest even), the first in the low half.
__device__ __forceinline__ uint32_t pack_f16x2(float lo, float hi) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)lo) | ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)hi) << 16);
}

// NW waves per workgroup: 2 rows of NW / 2 waves, each wave a 64 x (256 / NW)
// part of the tile (32 x 32 blocks 2 x NBN).  In a diagonal tile a block whose
// columns lie above its rows is skipped, and a wave with no block left only
// converts and keeps the barriers.
template <int EK, bool DIAG, int NW>
__device__ __forceinline__ void mfma_tile_128_cvt(const XArgs& a, int8_t* lds, int ch, int split, int I, int J) {
  constexpr int EKM = EK == kElemF16Cvt ? kElemF16 : kElemF8;   // the MFMA stage's element kind
  static_assert(NW == 4 || NW == 8, "4 or 8 waves");
  constexpr int NT = NW * 64;                     // threads
  constexpr int NWN = NW / 2;                     // waves across the tile's columns
  constexpr int NBN = 4 / NWN;                    // 32-column blocks per wave
  constexpr int BT = 128;
  constexpr int PANEL = BT * kMKC;                // bytes per operand per stage
  constexpr int STAGE = PANEL * (DIAG ? 1 : 2);
  constexpr int NOP = DIAG ? 1 : 2;
  constexpr int SB = EKM == kElemF16 ? 4 : 2;     // staged bytes per complex sample
  constexpr int SPS = kMKC / SB;                  // samples per row per stage
  constexpr int NF = SPS / 2;                     // float4 (two samples) per row per stage
  constexpr int L = BT * NF / NT;                 // float4 per thread per operand per stage
  using Acc = typename MAcc<EKM>::T;
  // register stages in flight: FP16 holds 2 float4 per thread and operand per
  // stage, so 4 stages fit at two waves per SIMD (2.6 % faster on C4 than 3);
  // FP8 holds 8 and keeps kPF.
  constexpr int PF = EKM == kElemF16 ? 4 : kPF;

  const float* __restrict__ xc = reinterpret_cast<const float*>(static_cast<const int8_t*>(a.x) + (int64_t)ch * a.ch_stride_b);
  const int64_t k0 = (int64_t)split * a.k_split_bytes;
  const int64_t k1 = min(a.k_bytes, k0 + a.k_split_bytes);
  const int n_st = k1 > k0 ? (int)((k1 - k0 + kMKC - 1) / kMKC) : 0;
  const int64_t t0 = k0 / SB, t1 = k1 / SB;        // sample range of the pass
  const int64_t rsf = a.row_stride_b / 4;          // floats between rows (row_stride_b: float32 bytes)
  // float4 loads when every row starts 16-byte aligned, else float2 loads
  const bool a16 = ((reinterpret_cast<uintptr_t>(xc) | (uintptr_t)a.row_stride_b) & 15) == 0;
  float sc = 1.f;
  if constexpr (EKM == kElemF8) sc = e4m3_scale(__uint_as_float(a.m_bits[ch]));

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / NWN, wn = wave % NWN;

  // This thread's loads: row q_row[q] (of 128), float4 f = q_f[q] of the
  // row's stage; LDS byte offset of the converted bytes within a panel.
  const float* src[2][L];
  int q_f[L], q_lds[L];
#pragma unroll
  for (int q = 0; q < L; ++q) {
    const int idx = tid + NT * q;
    const int r = idx / NF, f = idx % NF;
    const int kb = f * 2 * SB;                   // K byte of the float4's first sample
    q_f[q] = f;
    q_lds[q] = r * kMKC + 16 * ((kb >> 4) ^ swz(r)) + (kb & 15);
    src[0][q] = xc + (int64_t)min(I * BT + r, a.n_in - 1) * rsf;
    src[1][q] = xc + (int64_t)min(J * BT + r, a.n_in - 1) * rsf;
  }
  float4 R[PF][NOP][L];
  auto gload = [&](auto S, int st) {
    constexpr int sl = decltype(S)::value;
    const int64_t tb = t0 + (int64_t)st * SPS;
#pragma unroll
    for (int o = 0; o < NOP; ++o)
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const int64_t t = tb + 2 * q_f[q];
        const float* g = src[o][q] + t * 2;
        float4 v;
        if (t + 2 <= t1) {
          if (a16) {
            v = *reinterpret_cast<const float4*>(g);
          } else {
            const float2 u0 = reinterpret_cast<const float2*>(g)[0];
            const float2 u1 = reinterpret_cast<const float2*>(g)[1];
            v = make_float4(u0.x, u0.y, u1.x, u1.y);
          }
        } else {
          v = make_float4(0.f, 0.f, 0.f, 0.f);
          if (t < t1) {
            v.x = g[0];
            v.y = g[1];
          }
        }
        R[sl][o][q] = v;
      }
  };
  auto cvt_store = [&](auto S, int buf) {
    constexpr int sl = decltype(S)::value;
    int8_t* base = lds + buf * STAGE;
#pragma unroll
    for (int o = 0; o < NOP; ++o)
#pragma unroll
      for (int q = 0; q < L; ++q) {
        const float4 v = R[sl][o][q];
        int8_t* d = base + o * PANEL + q_lds[q];
        if constexpr (EKM == kElemF16) {
          *reinterpret_cast<uint2*>(d) = make_uint2(pack_f16x2(v.x, v.y), pack_f16x2(v.z, v.w));
        } else {
          int x = __builtin_amdgcn_cvt_pk_fp8_f32(sc * v.x, sc * v.y, 0, false);
          x = __builtin_amdgcn_cvt_pk_fp8_f32(sc * v.z, sc * v.w, x, true);
          *reinterpret_cast<int*>(d) = x;
        }
      }
  };

  Acc vr[2][NBN], vi[2][NBN];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < NBN; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        vr[m][n][r] = 0;
        vi[m][n][r] = 0;
      }

  const int frow = lane & 31;
  const int g = lane >> 5;
  auto read = [&](int buf, v4i (&af)[2][2], v4i (&bf)[NBN][2]) {
    const int8_t* As = lds + buf * STAGE;
    const int8_t* Bs = DIAG ? As : As + PANEL;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int cidx = 2 * h + g;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int r = wm * 64 + m * 32 + frow;
        af[m][h] = *reinterpret_cast<const v4i*>(As + r * kMKC + 16 * (cidx ^ swz(r)));
      }
#pragma unroll
      for (int n = 0; n < NBN; ++n) {
        const int r = (wn * NBN + n) * 32 + frow;
        bf[n][h] = *reinterpret_cast<const v4i*>(Bs + r * kMKC + 16 * (cidx ^ swz(r)));
      }
    }
  };
  // 32 x 32 block (m, n) of this wave: rows 2 wm + m, columns wn NBN + n (in
  // blocks); above the diagonal of a diagonal tile it is skipped.
  auto skip = [&](int m, int n) { return DIAG && wn * NBN + n > 2 * wm + m; };
  const bool idle = DIAG && wn * NBN > 2 * wm + 1;   // every block of the wave skipped
  auto compute = [&](const v4i (&af)[2][2], const v4i (&bf)[NBN][2]) {
    v4i ra[2][2];
    if constexpr (EKM == kElemF8) {
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < NBN; ++n)
          if (!skip(m, n)) mfma64<EKM>(af[m], bf[n], vr[m][n]);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) ra[m][h] = rotm4<EKM>(af[m][h]);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < NBN; ++n)
          if (!skip(m, n)) mfma64<EKM>(ra[m], bf[n], vi[m][n]);
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < NBN; ++n)
            if (!skip(m, n)) mfma16<EKM>(af[m][h], bf[n][h], vr[m][n]);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) ra[m][h] = rotm4<EKM>(af[m][h]);
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
          for (int n = 0; n < NBN; ++n)
            if (!skip(m, n)) mfma16<EKM>(ra[m][h], bf[n][h], vi[m][n]);
    }
  };

  using S0 = std::integral_constant<int, 0>;
  static_assert(PF == 3 || PF == 4, "the prologue and the unrolled main loop below are written for 3 or 4 slots");
  // prologue: stages 0 .. PF - 1 in flight (slot p holds stage p)
  if (0 < n_st) gload(S0{}, 0);
  if (1 < n_st) gload(std::integral_constant<int, 1>{}, 1);
  if (2 < n_st) gload(std::integral_constant<int, 2>{}, 2);
  if constexpr (PF == 4) {
    if (3 < n_st) gload(std::integral_constant<int, PF == 4 ? 3 : 0>{}, 3);
  }
  if (n_st > 0) {
    cvt_store(S0{}, 0);
    if (PF < n_st) gload(S0{}, PF);
  }
  __syncthreads();
  // Stage st lives in register slot st % PF; iteration st converts stage
  // st + 1 (freeing its slot) and refills that slot with stage st + 1 + PF.
  auto step = [&](auto U, int st) {
    constexpr int u = decltype(U)::value;
    constexpr int nx = (u + 1) % PF;
    v4i af[2][2], bf[NBN][2];
    if (!idle) read(st & 1, af, bf);
    if (st + 1 < n_st) {
      cvt_store(std::integral_constant<int, nx>{}, (st + 1) & 1);   // the buffer last read in stage st - 1
      if (st + 1 + PF < n_st) gload(std::integral_constant<int, nx>{}, st + 1 + PF);
    }
    if (!idle) compute(af, bf);
    __syncthreads();
  };
  for (int st0 = 0; st0 < n_st; st0 += PF) {
    step(std::integral_constant<int, 0>{}, st0);
    if (st0 + 1 < n_st) step(std::integral_constant<int, 1>{}, st0 + 1);
    if (st0 + 2 < n_st) step(std::integral_constant<int, 2>{}, st0 + 2);
    if constexpr (PF == 4) {
      if (st0 + 3 < n_st) step(std::integral_constant<int, PF == 4 ? 3 : 0>{}, st0 + 3);
    }
  }
  if (idle) return;

  // Epilogue (32 x 32 accumulator layout: register r of lane l holds row
  // 8*(r/4) + 4*(l/32) + r%4, column l%32).  FP8 sums are s_c^2 V exactly.
  const float scale = EKM == kElemF8 ? 1.f / (sc * sc) : 1.f;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < NBN; ++n) {
      if (skip(m, n)) continue;
      const int j = J * BT + (wn * NBN + n) * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = I * BT + wm * 64 + m * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (i < a.n_in && j <= i) {
          const int64_t off = (int64_t)split * a.out_split_stride + (int64_t)ch * a.n_products + tri_index(i, j);
          float2* pp = static_cast<float2*>(a.out) + off;
          const float re = vr[m][n][r] * scale;
          const float im = (i == j) ? 0.f : vi[m][n][r] * scale;
          if (a.accumulate) {
            float2 o = *pp;
            o.x += re;
            o.y += im;
            *pp = o;
          } else {
            *pp = make_float2(re, im);
          }
        }
      }
    }
}

// CI4 samples (one byte per complex sample: re in bits 7..4, im in bits 3..0,
// two's complement nibbles, the "1-byte" mode of Sec. 5) are unpacked in
// registers into int8 operands scaled by 16: the byte's high nibble with the
// low nibble cleared is 16 re, and the low nibble shifted up is 16 im, both
// exact in int8 for |re|, |im| <= 7.  Operand bytes run [16 re of 4 samples,
// 16 im of the same 4, 16 re of the next 4, 16 im of those]; the same order
// in A and B makes A B^T = sum (re re' + im im') = Re V (times 256).
constexpr uint32_t kHiNib = 0xF0F0F0F0u;
__device__ __forceinline__ v4i ci4_plain(int w0, int w1) {
  const uint32_t u0 = (uint32_t)w0, u1 = (uint32_t)w1;
  return v4i{(int)(u0 & kHiNib), (int)((u0 << 4) & kHiNib), (int)(u1 & kHiNib), (int)((u1 << 4) & kHiNib)};
}
// -16 re per byte of a high-nibble word: flip the nibble and add 1 in it; a
// carry out of a byte (re = 0) lands in the next byte's clear low nibble and
// is masked off.
__device__ __forceinline__ uint32_t neg_hi_nibbles(uint32_t x) { return ((x ^ kHiNib) + 0x10101010u) & kHiNib; }
// Operands of -iA = (im, -re) in the same byte order: A' B^T = sum (im re' -
// re im') = Im V (times 256).
__device__ __forceinline__ v4i ci4_rotm(int w0, int w1) {
  const uint32_t u0 = (uint32_t)w0, u1 = (uint32_t)w1;
  return v4i{(int)((u0 << 4) & kHiNib), (int)neg_hi_nibbles(u0 & kHiNib), (int)((u1 << 4) & kHiNib),
             (int)neg_hi_nibbles(u1 & kHiNib)};
}

// int8 variant of mfma_tile_128 on v_mfma_i32_16x16x64_i8: the same staging,
// pipeline and 64 x 64 wave tile, as 4 x 4 blocks of 16 x 16.  Each fragment
// read is one contiguous 1 KB of LDS (16 rows x 64 bytes), and the MFMA moves
// half the accumulator registers per multiply-accumulate of the 32 x 32 x 32
// form; measured on the MI355X it runs the C3 integration ≈4 % faster (the
// clock under load rises from ≈1.67 to ≈1.87 GHz).  A diagonal wave skips the
// 6 strictly upper 16 x 16 blocks of its quarter.
template <int EK, bool DIAG>
__device__ __forceinline__ void mfma_tile_128_i8(const XArgs& a, int8_t* lds, int ch, int split, int I, int J) {
  constexpr int BT = 128;
  constexpr int PANEL = BT * kMKC;           // bytes per operand per stage
  constexpr int STAGE = PANEL * (DIAG ? 1 : 2);
  constexpr int QPW = BT / 16 / 4;           // 1 KB load instructions per operand per wave
  constexpr int LPW = QPW * (DIAG ? 1 : 2);  // load instructions per wave per stage
  static_assert(EK == kElemI8 || EK == kElemCI4, "16 x 16 x 64 tile is the int8 engine");

  const int8_t* __restrict__ xc = static_cast<const int8_t*>(a.x) + (int64_t)ch * a.ch_stride_b;
  const int64_t k0 = (int64_t)split * a.k_split_bytes;
  const int64_t k1 = min(a.k_bytes, k0 + a.k_split_bytes);
  const int n_st = k1 > k0 ? (int)((k1 - k0 + kMKC - 1) / kMKC) : 0;
  const int64_t last = ((k1 - 1) >> 4) << 4;   // last valid 16-byte chunk start
  // Stages whose 64 bytes all lie in [k0, k1) and whose offsets fit 32 bits.
  const int n_fast = a.row_stride_b < (int64_t(1) << 24) ? (int)((k1 - k0) / kMKC) : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  // This lane's part of each load instruction: LDS row lrow (of 16), chunk p.
  const int lrow = lane >> 2, p = lane & 3;
  const int8_t* gA[QPW];
  const int8_t* gB[QPW];
  uint32_t oA[QPW], oB[QPW];
  int rowq[QPW];
  const int8_t* tA = xc + (int64_t)(I * BT) * a.row_stride_b + k0;
  const int8_t* tB = xc + (int64_t)(J * BT) * a.row_stride_b + k0;
#pragma unroll
  for (int q = 0; q < QPW; ++q) {
    const int r = (wave * QPW + q) * 16 + lrow;    // tile row
    rowq[q] = r;
    const int c = p ^ swz(r);                      // global chunk this lane fetches
    const int ra = min(I * BT + r, a.n_in - 1);
    const int rb = min(J * BT + r, a.n_in - 1);
    gA[q] = xc + (int64_t)ra * a.row_stride_b + 16 * c;
    gB[q] = xc + (int64_t)rb * a.row_stride_b + 16 * c;
    oA[q] = (uint32_t)((int64_t)(ra - I * BT) * a.row_stride_b + 16 * c);
    oB[q] = (uint32_t)((int64_t)(rb - J * BT) * a.row_stride_b + 16 * c);
  }
  auto issue = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE + wave * QPW * 1024;
    if (st < n_fast) {
      const int8_t* ga = tA + st * kMKC;
      const int8_t* gb = tB + st * kMKC;
#pragma unroll
      for (int q = 0; q < QPW; ++q) {
        __builtin_amdgcn_global_load_lds(ga + oA[q], base + q * 1024, 16, 0, 0);
        if (!DIAG) __builtin_amdgcn_global_load_lds(gb + oB[q], base + q * 1024 + PANEL, 16, 0, 0);
      }
    } else {
      const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
      for (int q = 0; q < QPW; ++q) {
        const int c = p ^ swz(rowq[q]);
        const int64_t kk = kb + 16 * c;
        const int64_t off = (kk <= last ? kb : last - 16 * c);   // keep the 16 bytes inside the row
        __builtin_amdgcn_global_load_lds(gA[q] + off, base + q * 1024, 16, 0, 0);
        if (!DIAG) __builtin_amdgcn_global_load_lds(gB[q] + off, base + q * 1024 + PANEL, 16, 0, 0);
      }
    }
  };
  // Zero / mask the chunks of stage st that reach past k1 (only the last stage).
  auto fix_tail = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE;
    const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
    for (int q = 0; q < QPW; ++q) {
      const int c = p ^ swz(rowq[q]);
      const int64_t kk = kb + 16 * c;
      if (kk + 16 > k1) {
        const int64_t valid = k1 - kk;
#pragma unroll
        for (int op = 0; op < (DIAG ? 1 : 2); ++op) {
          v4i* cell = reinterpret_cast<v4i*>(base + op * PANEL + (wave * QPW + q) * 1024 + lane * 16);
          v4i v = *cell;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t lo = 4 * w;
            const int keep = valid >= lo + 4 ? 4 : (valid > lo ? (int)(valid - lo) : 0);
            const uint32_t m = keep >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keep)) - 1u);
            v[w] = (int)((uint32_t)v[w] & m);
          }
          *cell = v;
        }
      }
    }
  };

  v4i vr[4][4], vi[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      vr[m][n] = v4i{0, 0, 0, 0};
      vi[m][n] = v4i{0, 0, 0, 0};
    }

#pragma unroll
  for (int s = 0; s < kMNS - 1; ++s)
    if (s < n_st) issue(s);

  const bool tail = (k1 - k0) % kMKC != 0;
  // Wait for this wave's loads of stage st (later stages stay in flight),
  // mask the K tail, and make stage st visible to all waves.  A plain
  // s_barrier: a fenced one would also drain the later stages' loads.
  auto arrive = [&](int st) {
    const int ahead = min(kMNS - 2, n_st - 1 - st);
    if (ahead >= 2) wait_vmcnt<2 * LPW>();
    else if (ahead == 1) wait_vmcnt<LPW>();
    else wait_vmcnt<0>();
    if (tail && st == n_st - 1) fix_tail(st);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    asm volatile("s_barrier" ::: "memory");
  };
  // 16 x 16 x 64 fragments: lane l reads row (l % 16) of a 16-row block,
  // 16-byte chunk l / 16 (the whole 64-byte stage row across 4 lanes).
  auto read = [&](int st, v4i (&af)[4], v4i (&bf)[4]) {
    const int8_t* As = lds + (st % kMNS) * STAGE;
    const int8_t* Bs = DIAG ? As : As + PANEL;
    const int c = lane >> 4;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = wm * 64 + m * 16 + (lane & 15);
      af[m] = *reinterpret_cast<const v4i*>(As + r * kMKC + 16 * (c ^ swz(r)));
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int r = wn * 64 + n * 16 + (lane & 15);
      bf[n] = *reinterpret_cast<const v4i*>(Bs + r * kMKC + 16 * (c ^ swz(r)));
    }
  };
  auto compute = [&](auto sk, const v4i (&af)[4], const v4i (&bf)[4]) {
    constexpr bool SK = decltype(sk)::value;
    if constexpr (EK != kElemCI4) {   // CI4 stages run through compute_ci4
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          if (!(SK && n > m)) vr[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[m], bf[n], vr[m][n], 0, 0, 0);
      v4i ra[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) ra[m] = rotm4<kElemI8>(af[m]);
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
          if (!(SK && n > m)) vi[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ra[m], bf[n], vi[m][n], 0, 0, 0);
    }
  };

  if (n_st > 0) {
    arrive(0);
    if (kMNS - 1 < n_st) issue(kMNS - 1);
  }
  // In a diagonal tile the wave of the strictly upper 64 x 64 quarter only
  // loads its share of the panel and keeps the barriers.
  if (DIAG && wm < wn) {
    for (int s = 0; s + 1 < n_st; ++s) {
      arrive(s + 1);
      if (s + kMNS < n_st) issue(s + kMNS);
    }
    return;
  }
  // CI4: a stage's 16 packed samples per lane feed two K steps (dwords 0-1
  // of every A and B fragment the first, 2-3 the second).  Each step's
  // operands are unpacked just before its 32 MFMAs; once the second step's
  // are unpacked the packed registers take the next stage's LDS reads, which
  // then run under the second step's MFMAs.
  auto unpack_ci4 = [&](int h, const v4i (&pa)[4], const v4i (&pb)[4], v4i (&ua)[4], v4i (&ub)[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      ua[m] = ci4_plain(pa[m][2 * h], pa[m][2 * h + 1]);
      ub[m] = ci4_plain(pb[m][2 * h], pb[m][2 * h + 1]);
    }
  };
  auto compute_ci4 = [&](auto sk, const v4i (&ua)[4], const v4i (&ub)[4]) {
    constexpr bool SK = decltype(sk)::value;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < 4; ++n)
        if (!(SK && n > m)) vr[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ua[m], ub[n], vr[m][n], 0, 0, 0);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      // -iA = (im, -re): the operand's im words, and its re words negated
      const v4i a = ua[m];
      const v4i ra = {a[1], (int)neg_hi_nibbles((uint32_t)a[0]), a[3], (int)neg_hi_nibbles((uint32_t)a[2])};
#pragma unroll
      for (int n = 0; n < 4; ++n)
        if (!(SK && n > m)) vi[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ra, ub[n], vi[m][n], 0, 0, 0);
    }
  };
  auto run_ci4 = [&](auto sk) {
    constexpr int NM = (DIAG && decltype(sk)::value) ? 20 : 32;   // MFMAs per K step
    v4i pa[4], pb[4], ua[4], ub[4];
    if (n_st > 0) read(0, pa, pb);
    for (int s = 0; s < n_st; ++s) {
      unpack_ci4(0, pa, pb, ua, ub);
      compute_ci4(sk, ua, ub);
      unpack_ci4(1, pa, pb, ua, ub);
      if (s + 1 < n_st) {
        arrive(s + 1);
        if (s + kMNS < n_st) issue(s + kMNS);
        read(s + 1, pa, pb);
      }
      compute_ci4(sk, ua, ub);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, NM - 8, 0);
    }
  };
  auto run = [&](auto sk) {
    constexpr int NM = (DIAG && decltype(sk)::value) ? 20 : 32;   // MFMAs per stage
    v4i af0[4], bf0[4], af1[4], bf1[4];
    if (n_st > 0) read(0, af0, bf0);
    for (int s = 0; s + 1 < n_st; ++s) {
      arrive(s + 1);
      if (s + kMNS < n_st) issue(s + kMNS);
      read(s + 1, af1, bf1);
      compute(sk, af0, bf0);
#pragma unroll
      for (int q = 0; q < (NM < 8 ? NM : 8); ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      }
      if constexpr (NM > 8) __builtin_amdgcn_sched_group_barrier(0x008, NM - 8, 0);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        af0[m] = af1[m];
        bf0[m] = bf1[m];
      }
    }
    if (n_st > 0) compute(sk, af0, bf0);
  };
  if constexpr (EK == kElemCI4) {
    if (DIAG && wm == wn) run_ci4(std::true_type{});
    else run_ci4(std::false_type{});
  } else {
    if (DIAG && wm == wn) run(std::true_type{});
    else run(std::false_type{});
  }

  // Epilogue.  16 x 16 accumulator layout: register r of lane l holds row
  // 4*(l/16) + r, column l%16.
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      const int j = J * BT + wn * 64 + n * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * BT + wm * 64 + m * 16 + 4 * (lane >> 4) + r;
        if (i < a.n_in && j <= i) {
          const int64_t off = (int64_t)split * a.out_split_stride + (int64_t)ch * a.n_products + tri_index(i, j);
          int2* pp = static_cast<int2*>(a.out) + off;
          // CI4 operands are 16 x the sample parts: the sums are 256 V exactly
          const int re = EK == kElemCI4 ? (vr[m][n][r] >> 8) : vr[m][n][r];
          const int im = (i == j) ? 0 : (EK == kElemCI4 ? (vi[m][n][r] >> 8) : vi[m][n][r]);
          if (a.accumulate) {
            int2 o = *pp;
            o.x += re;
            o.y += im;
            *pp = o;
          } else {
            *pp = make_int2(re, im);
          }
        }
      }
    }
}

template <int EK>
__global__ __launch_bounds__(256, 2) void xeng_mfma_128_kernel(XArgs a) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[kMNS * 2 * 128 * kMKC];
  const int64_t slot = blockIdx.x / kNumXcd;
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if (slot >= a.per_xcd || item >= a.n_items) return;
  int ch, split, I, J;
  item_decode(a, item, ch, split, I, J);
  if constexpr (EK == kElemI8 || EK == kElemCI4) {
    if (I == J) mfma_tile_128_i8<EK, true>(a, lds, ch, split, I, J);
    else mfma_tile_128_i8<EK, false>(a, lds, ch, split, I, J);
  } else {
    if (I == J) mfma_tile_128<EK, true>(a, lds, ch, split, I, J);
    else mfma_tile_128<EK, false>(a, lds, ch, split, I, J);
  }
}

// Waves per workgroup of the converting engines (one workgroup per CU).  FP16:
// 8 (two per SIMD, 64 x 32 wave parts, 177 VGPRs), 8 % faster on C4 than 4
// waves of 64 x 64.  FP8 stages twice the samples per row and would spill
// with 8, so it keeps 4 (measured slower with 8).
template <int EK>
constexpr int cvt_waves() { return EK == kElemF16Cvt ? 8 : 4; }

template <int EK>
__global__ __launch_bounds__(cvt_waves<EK>() * 64, 1) void xeng_cvt_128_kernel(XArgs a) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[2 * 2 * 128 * kMKC];
  const int64_t slot = blockIdx.x / kNumXcd;
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if (slot >= a.per_xcd || item >= a.n_items) return;
  int ch, split, I, J;
  item_decode(a, item, ch, split, I, J);
  if (I == J) mfma_tile_128_cvt<EK, true, cvt_waves<EK>()>(a, lds, ch, split, I, J);
  else mfma_tile_128_cvt<EK, false, cvt_waves<EK>()>(a, lds, ch, split, I, J);
}

// FP32 matrix-core tile: the 64-row tile of mfma_tile (same staging,
// pipeline and swizzle), but each wave's 32 x 32 quadrant runs as 2 x 2
// blocks of v_mfma_f32_16x16x4_f32.  A lane reads one 16-byte chunk (two
// complex samples) of its block row per stage -- row lane % 16, chunk lane /
// 16 -- and instruction q takes float q of it from A and from B, so the 16
// K elements of the stage enter once each, in the same place for both.  In a
// diagonal tile the quadrant waves skip their strictly upper 16 x 16 block:
// 2560 products computed per 2080 needed at 64 inputs, against 3072 with
// 32 x 32 blocks.
typedef float v4f __attribute__((ext_vector_type(4)));

template <bool DIAG>
__device__ __forceinline__ void mfma_tile_f32(const XArgs& a, int8_t* lds, int ch, int split, int I, int J) {
  constexpr int BT = 64;
  constexpr int PANEL = BT * kMKC;
  constexpr int STAGE = PANEL * (DIAG ? 1 : 2);
  constexpr int QPW = BT / 16 / 4;
  constexpr int LPW = QPW * (DIAG ? 1 : 2);

  const int8_t* __restrict__ xc = static_cast<const int8_t*>(a.x) + (int64_t)ch * a.ch_stride_b;
  const int64_t k0 = (int64_t)split * a.k_split_bytes;
  const int64_t k1 = min(a.k_bytes, k0 + a.k_split_bytes);
  const int n_st = k1 > k0 ? (int)((k1 - k0 + kMKC - 1) / kMKC) : 0;
  const int64_t last = ((k1 - 1) >> 4) << 4;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool wave_idle = DIAG && (wm < wn);
  const bool quad_diag = DIAG && (wm == wn);

  const int lrow = lane >> 2, p = lane & 3;
  const int8_t* gA[QPW];
  const int8_t* gB[QPW];
  int rowq[QPW];
#pragma unroll
  for (int q = 0; q < QPW; ++q) {
    const int r = (wave * QPW + q) * 16 + lrow;
    rowq[q] = r;
    const int c = p ^ swz(r);
    gA[q] = xc + (int64_t)min(I * BT + r, a.n_in - 1) * a.row_stride_b + 16 * c;
    if (!DIAG) gB[q] = xc + (int64_t)min(J * BT + r, a.n_in - 1) * a.row_stride_b + 16 * c;
  }
  auto issue = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE;
    const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
    for (int q = 0; q < QPW; ++q) {
      const int c = p ^ swz(rowq[q]);
      const int64_t kk = kb + 16 * c;
      const int64_t off = (kk <= last ? kb : last - 16 * c);
      int8_t* dst = base + (wave * QPW + q) * 1024;
      __builtin_amdgcn_global_load_lds(gA[q] + off, dst, 16, 0, 0);
      if (!DIAG) __builtin_amdgcn_global_load_lds(gB[q] + off, dst + PANEL, 16, 0, 0);
    }
  };
  auto fix_tail = [&](int st) {
    int8_t* base = lds + (st % kMNS) * STAGE;
    const int64_t kb = k0 + (int64_t)st * kMKC;
#pragma unroll
    for (int q = 0; q < QPW; ++q) {
      const int c = p ^ swz(rowq[q]);
      const int64_t kk = kb + 16 * c;
      if (kk + 16 > k1) {
        const int64_t valid = k1 - kk;
#pragma unroll
        for (int op = 0; op < (DIAG ? 1 : 2); ++op) {
          v4i* cell = reinterpret_cast<v4i*>(base + op * PANEL + (wave * QPW + q) * 1024 + lane * 16);
          v4i v = *cell;
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int64_t lo = 4 * w;
            const int keep = valid >= lo + 4 ? 4 : (valid > lo ? (int)(valid - lo) : 0);
            const uint32_t m = keep >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keep)) - 1u);
            v[w] = (int)((uint32_t)v[w] & m);
          }
          *cell = v;
        }
      }
    }
  };

  v4f vr[2][2], vi[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      vr[m][n] = v4f{0.f, 0.f, 0.f, 0.f};
      vi[m][n] = v4f{0.f, 0.f, 0.f, 0.f};
    }

#pragma unroll
  for (int s = 0; s < kMNS - 1; ++s)
    if (s < n_st) issue(s);

  const int frow = lane & 15;
  const int c4 = lane >> 4;
  const bool tail = (k1 - k0) % kMKC != 0;
  for (int s = 0; s < n_st; ++s) {
    const int ahead = min(kMNS - 2, n_st - 1 - s);
    if (ahead >= 2) wait_vmcnt<2 * LPW>();
    else if (ahead == 1) wait_vmcnt<LPW>();
    else wait_vmcnt<0>();
    if (tail && s == n_st - 1) {
      fix_tail(s);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
    asm volatile("s_barrier" ::: "memory");
    if (s + kMNS - 1 < n_st) issue(s + kMNS - 1);
    if (!wave_idle) {
      const int8_t* As = lds + (s % kMNS) * STAGE;
      const int8_t* Bs = DIAG ? As : As + PANEL;
      v4i af[2], bf[2], bj[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int r = wm * 32 + m * 16 + frow;
        af[m] = *reinterpret_cast<const v4i*>(As + r * kMKC + 16 * (c4 ^ swz(r)));
      }
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const int r = wn * 32 + n * 16 + frow;
        bf[n] = *reinterpret_cast<const v4i*>(Bs + r * kMKC + 16 * (c4 ^ swz(r)));
        bj[n] = rot4<kElemF32>(bf[n]);
      }
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          if (quad_diag && m < n) continue;   // strictly upper 16 x 16 block
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            vr[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(__int_as_float(af[m][q]), __int_as_float(bf[n][q]),
                                                            vr[m][n], 0, 0, 0);
            vi[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(__int_as_float(af[m][q]), __int_as_float(bj[n][q]),
                                                            vi[m][n], 0, 0, 0);
          }
        }
    }
  }

  if (wave_idle) return;
  // Epilogue.  16 x 16 accumulator layout: register r of lane l holds row
  // 4*(l/16) + r, column l%16.
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      if (quad_diag && m < n) continue;
      const int j = J * BT + wn * 32 + n * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * BT + wm * 32 + m * 16 + 4 * (lane >> 4) + r;
        if (i < a.n_in && j <= i) {
          const int64_t off = (int64_t)split * a.out_split_stride + (int64_t)ch * a.n_products + tri_index(i, j);
          float2* pp = static_cast<float2*>(a.out) + off;
          const float re = vr[m][n][r];
          const float im = (i == j) ? 0.f : vi[m][n][r];
          if (a.accumulate) {
            float2 o = *pp;
            o.x += re;
            o.y += im;
            *pp = o;
          } else {
            *pp = make_float2(re, im);
          }
        }
      }
    }
}

// Diagonal or off-diagonal tile of the BT-row engine (one instantiation site
// for every kernel that runs BT-row tiles).
template <int EK, int BT>
__device__ __forceinline__ void mfma_tile_any(const XArgs& a, int8_t* lds, int ch, int split, int I, int J) {
  if constexpr (EK == kElemF32) {
    static_assert(BT == 64, "the FP32 matrix-core engine runs 64-row tiles");
    if (I == J) mfma_tile_f32<true>(a, lds, ch, split, I, J);
    else mfma_tile_f32<false>(a, lds, ch, split, I, J);
  } else {
    if (I == J) mfma_tile<EK, BT, true>(a, lds, ch, split, I, J);
    else mfma_tile<EK, BT, false>(a, lds, ch, split, I, J);
  }
}

template <int EK, int BT>
__global__ __launch_bounds__(256, 2) void xeng_mfma_kernel(XArgs a) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[kMNS * 2 * BT * kMKC];
  const int64_t slot = blockIdx.x / kNumXcd;
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if (slot >= a.per_xcd || item >= a.n_items) return;
  int ch, split, I, J;
  item_decode(a, item, ch, split, I, J);
  mfma_tile_any<EK, BT>(a, lds, ch, split, I, J);
}

// Serving: a device queue of integration jobs shared by persistent grids.
// The host scheduler publishes each admitted job in a slot (its sample and
// output pointers and shape) and lists the slots whose jobs have unclaimed
// items; every workgroup of the running serving grid claims work items --
// (channel, 128-row tile) pairs -- from the listed jobs in turn (round robin
// over the jobs: a small job is not queued behind a large one, and the claims
// of the grid's workgroups spread over the jobs' counters), runs the tile
// over all of the job's samples, and counts it done.  The workgroup that claims a job's last item reports it to
// the host (which then lists the job no more); the workgroup that finishes
// the job's last item writes the job's completion word in host memory.
//
// A grid ends as a whole: once no workgroup has claimed an item for
// idle_ticks of the 100 MHz wall clock, the first workgroup to notice closes
// the grid (it raises `closing` to the grid's generation and tells the host),
// and from then on no workgroup of that generation claims again; each exits
// after its current tile.  So a running grid never thins out to a few
// workgroups that would then carry new work alone; work published after the
// close waits for the next grid, which the scheduler launches at full size.
__device__ __forceinline__ uint64_t sys_load64(const void* p) {
  return __hip_atomic_load(static_cast<const uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Thread 0: claim one item, or return -1 when the grid has closed (or this
// workgroup has polled max_polls times without work).
__device__ int serve_claim(const ServeQueue& q, uint64_t* claimed) {
  for (int poll = 0; poll < q.max_polls; ++poll) {
    if (__hip_atomic_load(q.closing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= q.gen) return -1;
    const int n = __hip_atomic_load(q.active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    if (n > 0 && n <= q.n_slots) {
      const uint32_t r = __hip_atomic_fetch_add(q.rr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (int a = 0; a < n; ++a) {
        const int s = __hip_atomic_load(q.active + 1 + (int)((r + (uint32_t)a) % (uint32_t)n), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_SYSTEM);
        if (s < 0 || s >= q.n_slots) continue;
        uint64_t* cw = q.claim + (size_t)s * (kServeLine / 2);
        const uint64_t lim = sys_load64(q.limit + (size_t)s * (kServeLine / 2));
        uint64_t w = __hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (w < lim) {
          if (__hip_atomic_compare_exchange_strong(cw, &w, w + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_fetch_max(q.last_claim, (uint64_t)wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            // the job's last item: tell the host, which then lists the job no more
            if (w + 1 == lim)
              __hip_atomic_store(q.host_claimed + (size_t)s * (kServeLine / 2) + 1, lim, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_SYSTEM);
            *claimed = w;
            return s;
          }
        }
      }
    }
    const uint64_t last = __hip_atomic_load(q.last_claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint64_t)wall_clock64() > last + q.idle_ticks) {
      uint32_t c = __hip_atomic_load(q.closing, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (c < q.gen && !__hip_atomic_compare_exchange_strong(q.closing, &c, q.gen, __ATOMIC_RELAXED,
                                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
      }
      if (c < q.gen) __hip_atomic_store(q.host_closing, q.gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      return -1;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  return -1;
}

// The job's arguments and the claimed item pass through the start of the
// tile's LDS buffer (one LDS object per kernel: a second one makes the
// compiler wait for every LDS-bound global load before each LDS read).
struct ServeClaim {
  ServeJob job;
  int32_t slot, item;
};

__global__ __launch_bounds__(256, 2) void xeng_serve_kernel(ServeQueue q) {
  __shared__ __attribute__((aligned(1024))) int8_t lds[kMNS * 2 * 128 * kMKC];
  static_assert(sizeof(ServeClaim) <= sizeof(lds), "claim record fits in the tile buffer");
  ServeClaim* sc = reinterpret_cast<ServeClaim*>(lds);
  if (threadIdx.x == 0)   // a new grid counts as activity: it lingers idle_ticks before it may close
    __hip_atomic_fetch_max(q.last_claim, (uint64_t)wall_clock64(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    __syncthreads();   // the previous tile's LDS reads are done
    if (threadIdx.x == 0) {
      uint64_t claimed = 0;
      const int slot = serve_claim(q, &claimed);
      if (slot >= 0) {
        const uint64_t* src = reinterpret_cast<const uint64_t*>(q.slots + slot);
        uint64_t* dst = reinterpret_cast<uint64_t*>(&sc->job);
        for (int k = 0; k < (int)(sizeof(ServeJob) / 8); ++k) dst[k] = sys_load64(src + k);
        sc->item = (int)(claimed - sc->job.base);
      }
      sc->slot = slot;
    }
    __syncthreads();
    const int slot = sc->slot;
    if (slot < 0) return;
    const XArgs a = sc->job.x;
    const int item = sc->item;
    uint32_t* const flag_word = sc->job.flag;
    const uint32_t flag_value = sc->job.flag_value;
    const uint64_t job_end = sc->job.base + (uint64_t)a.n_items;
    __syncthreads();   // everyone holds the claim before the tile reuses the buffer
    const int tile = item % a.n_tiles;
    const int ch = item / a.n_tiles;
    int I, J;
    tile_decode(tile, I, J);
    if (I == J) mfma_tile_128_i8<kElemI8, true>(a, lds, ch, 0, I, J);
    else mfma_tile_128_i8<kElemI8, false>(a, lds, ch, 0, I, J);
    __threadfence();   // this thread's part of the tile is visible device-wide
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t old = __hip_atomic_fetch_add(q.done + (size_t)slot * kServeLine, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
      if ((uint64_t)old + 1 == job_end) {
        __threadfence_system();
        __hip_atomic_store(flag_word, flag_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

hipError_t launch_xeng_mfma(const XArgs& a, int elem, int bt, hipStream_t s) {
  const int64_t grid = (int64_t)a.per_xcd * kNumXcd;
  if (grid <= 0) return hipSuccess;
  const dim3 g((unsigned)grid), b(256);
#define CORR_LAUNCH(EK, BT) hipLaunchKernelGGL((xeng_mfma_kernel<EK, BT>), g, b, 0, s, a)
#define CORR_LAUNCH_W2(EK) hipLaunchKernelGGL((xeng_mfma_128_kernel<EK>), g, b, 0, s, a)
  if (elem == kElemI8) {
    if (bt == 128) CORR_LAUNCH_W2(kElemI8); else CORR_LAUNCH(kElemI8, 64);
  } else if (elem == kElemF32) {
    CORR_LAUNCH(kElemF32, 64);   // 64-row tiles only
  } else if (elem == kElemCI4) {
    CORR_LAUNCH_W2(kElemCI4);   // 128-row tiles only
  } else if (elem == kElemF16Cvt) {   // 128-row tiles only
    hipLaunchKernelGGL((xeng_cvt_128_kernel<kElemF16Cvt>), g, dim3(cvt_waves<kElemF16Cvt>() * 64), 0, s, a);
  } else if (elem == kElemF8Cvt) {
    hipLaunchKernelGGL((xeng_cvt_128_kernel<kElemF8Cvt>), g, dim3(cvt_waves<kElemF8Cvt>() * 64), 0, s, a);
  } else if (elem == kElemF16) {
    if (bt == 128) CORR_LAUNCH_W2(kElemF16); else CORR_LAUNCH(kElemF16, 64);
  } else {
    if (bt == 128) CORR_LAUNCH_W2(kElemF8); else CORR_LAUNCH(kElemF8, 64);
  }
#undef CORR_LAUNCH
#undef CORR_LAUNCH_W2
  return hipGetLastError();
}

hipError_t launch_xeng_serve(const ServeQueue& q, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(xeng_serve_kernel, dim3((unsigned)grid), dim3(256), 0, s, q);
  return hipGetLastError();
}

int serve_blocks_per_cu() {
  int n = 0;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, xeng_serve_kernel, 256, 0) == hipSuccess ? n : 0;
}

}  // namespace corr
