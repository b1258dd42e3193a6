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
#include "fft_device.h"
#include "launch.h"

namespace corr {

constexpr int kFN = 256;          // FFT length
constexpr int kFCh = kFN / 2;     // channels kept
constexpr int kFBlk = 16;         // blocks per workgroup
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
  int32_t n_ig;            // input groups = ceil(n_in / inputs per workgroup)
  float scale;             // requantisation scale s
  float max_abs;
  int32_t vec_in;          // 1: n_in a multiple of, and volt aligned to, the inputs per workgroup
  int32_t vec_out;         // 1: t_offset % 8 == 0 and ring_stride % 8 == 0
  int64_t n_items;         // block groups (padded to a multiple of 4) x input groups
  int64_t per_xcd;         // ceil(n_items / 8)
  const float* pfb;        // filterbank coefficients h[p*256 + n], p < TAPS (TAPS > 1 only)
};

// Low bytes of four requantised values -> (b0, b1, b2, b3) of one word.
__device__ __forceinline__ uint32_t pack4(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3) {
  const uint32_t lo = __builtin_amdgcn_perm(b1, b0, 0x0c0c0400u);  // (b0.0, b1.0, 0, 0)
  const uint32_t hi = __builtin_amdgcn_perm(b3, b2, 0x04000c0cu);  // (0, 0, b2.0, b3.0)
  return lo | hi;
}

// Signed byte j of w as float.
template <int J>
__device__ __forceinline__ float sbyte(uint32_t w) {
  return (float)((int32_t)(w << (24 - 8 * J)) >> 24);
}

// One workgroup: 16 consecutive blocks x IN inputs (IN = 8 or 16, IN / 2
// pairs).  FFT slot f = tid / 16 (lanes l = tid % 16) owns block f: it loads
// its 16 samples x IN inputs straight into registers (IN bytes of each
// n_in-byte time row; more inputs per workgroup means fewer, fuller cache
// line requests) and runs one 256-point FFT per pair.  The exchange buffer
// S[f] is used by the 16 lanes of slot f only, all in one wave; O is the
// workgroup's corner turn for the current pair.
constexpr int kORow = 20;  // words per channel row of O (16 blocks + pad, 16-byte aligned rows)
constexpr int kPRow = kFN + 16;  // words per block of the filterbank window (a wave's 4 slots on distinct banks)
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// (re, im) bytes in the low 16 bits of v -> two binary16 in one word.
__device__ __forceinline__ uint32_t pair_f16(uint32_t v) {
  // exact: |values| <= 128
  return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(sbyte<0>(v), sbyte<1>(v)));
}

//
// TAPS > 1: polyphase filterbank in place of the plain transform (Sec. 6.1
// names it as the cure for the FFT's leakage): the input holds TAPS - 1
// more blocks than there are outputs, and block b's transform input is
// y_b[n] = sum_p h[p*256 + n] x[(b + p)*256 + n] (weighted overlap-add of
// TAPS consecutive blocks).  The workgroup's 16 +
// TAPS - 1 blocks are each loaded once, as a sliding window: slot f keeps its
// own block b0 + f in registers, and slots f < TAPS - 1 also block b0 + 16 +
// f.  For each pair the slots publish those blocks' two samples in an LDS
// window (in the exchange buffer's space) as binary16 pairs (exact for 8-bit
// integers), and slot f reads its TAPS taps (blocks f .. f + TAPS - 1) back
// from there at fixed offsets: one 4-byte read and two mixed-precision FMAs
// (binary16 operand, FP32 product and sum) per tap and sample.
template <int IN, int TAPS>
__global__ __launch_bounds__(256, 3) void fstage_kernel(FArgs a) {
  static_assert(IN == 8 || IN == 16, "inputs per workgroup");
  // (16 inputs with the filterbank need more than the 256 registers of two
  // workgroups per CU: measured spills)
  static_assert(TAPS == 1 || IN == 8, "the filterbank path takes 8 inputs per workgroup");
  constexpr int kW = IN / 4;  // words per sample and lane
  __shared__ __attribute__((aligned(16))) float2 S[kFFtPerRound][kFSRow * 16];  // 34 KB
  __shared__ __attribute__((aligned(16))) uint32_t O[kFCh][kORow];              // 10 KB
  __shared__ float2 tw[kFN];                                                     // 2 KB
  // filterbank coefficients by sample: hs[n] = (h[n], h[256 + n], h[512 + n], h[768 + n])
  __shared__ float4 hs[TAPS > 1 ? kFN : 1];                                      // 4 KB
  // Filterbank window: the current pair's samples of blocks b0 ..
  // b0+15+TAPS-1 (binary16 re, im per sample), 20 KB in the space of the
  // exchange buffer S, which the pair's transform uses only after a barrier
  // that follows the last read of the window.
  static_assert(TAPS == 1 || (kFBlk + TAPS - 1) * kPRow * 4 <= (int)sizeof(S), "the window fits in S");
  uint32_t* const P = reinterpret_cast<uint32_t*>(&S[0][0]);

  const int tid = threadIdx.x;
  // Items run through 4 consecutive block groups of one input group (the
  // four 32-byte pieces of each 128-byte ring line), then input groups, then
  // the next 4 block groups.  The XCD remap keeps each run of items on one
  // XCD (one L2): the n_ig workgroups of a block group read the same input
  // rows, and the four pieces of a line merge there before going to HBM.
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if ((int64_t)(blockIdx.x / kNumXcd) >= a.per_xcd || item >= a.n_items) return;
  const int64_t rest = item >> 2;
  const int ig = (int)(rest % a.n_ig);
  const int64_t b0 = ((rest / a.n_ig) * 4 + (item & 3)) * kFBlk;
  if (b0 >= a.n_blocks) return;
  const int i0 = ig * IN;
  const int f = tid >> 4;  // block of this FFT slot
  const int l = tid & 15;  // lane within the FFT
  const int64_t nb = min((int64_t)kFBlk, a.n_blocks - b0);

  // Samples t = l + 16 n2 of block b0 + f (and, filterbank, of block b0 + 16
  // + f for slots f < TAPS - 1, into wx), inputs i0..i0+IN-1 (zero outside;
  // a block is read when some output of this workgroup uses it).
  uint32_t w[16][kW];
  uint32_t wx[TAPS > 1 ? 16 : 1][kW];
  constexpr int kLoads = TAPS > 1 ? 2 : 1;
#pragma unroll
  for (int e = 0; e < kLoads; ++e) {
    const int j = e == 0 ? f : kFBlk + f;            // block offset from b0
    if (e == 1 && f >= TAPS - 1) break;
    const bool need = j < nb + TAPS - 1;
    uint32_t v[16][kW];
    if (a.vec_in && nb == kFBlk) {
      const int8_t* p = a.volt + ((b0 + j) * kFN + l) * a.n_in + i0;
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2) {
        const int8_t* q = p + (int64_t)n2 * 16 * a.n_in;
        if constexpr (IN == 16) {
          const uint4 u = *reinterpret_cast<const uint4*>(q);
          v[n2][0] = u.x; v[n2][1] = u.y; v[n2][2] = u.z; v[n2][3] = u.w;
        } else {
          const uint2 u = *reinterpret_cast<const uint2*>(q);
          v[n2][0] = u.x; v[n2][1] = u.y;
        }
      }
    } else {
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2) {
        const int64_t t = (b0 + j) * kFN + l + 16 * n2;
        const int8_t* p = a.volt + t * a.n_in + i0;
#pragma unroll
        for (int jj = 0; jj < kW; ++jj) {
          uint32_t u = 0;
          for (int q = 0; q < 4; ++q) {
            const int i = 4 * jj + q;
            if (need && i0 + i < a.n_in) u |= (uint32_t)(uint8_t)p[i] << (8 * q);
          }
          v[n2][jj] = u;
        }
      }
    }
    if (e == 0) {
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2)
#pragma unroll
        for (int jj = 0; jj < kW; ++jj) w[n2][jj] = v[n2][jj];
    } else if constexpr (TAPS > 1) {
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2)
#pragma unroll
        for (int jj = 0; jj < kW; ++jj) wx[n2][jj] = v[n2][jj];
    }
  }
  // Twiddle table W_256^m; a lane reads W_256^(l k2) for every round from it
  // (the first round's barrier orders these writes before the first read).
  tw[tid] = a.twiddle[tid];
  if constexpr (TAPS > 1) {
    static_assert(TAPS == 4, "hs holds four taps per sample");
    hs[tid] = make_float4(a.pfb[tid], a.pfb[kFN + tid], a.pfb[2 * kFN + tid], a.pfb[3 * kFN + tid]);
    __syncthreads();  // hs is complete
  }

  const float h = 0.5f * a.scale;  // the 1/2 of the two-for-one split folded into the scale
  const float lo = kRqMagic - a.max_abs, hi = kRqMagic + a.max_abs;
  // Mirror lookup: Z_{256-k} for k = l + 16 k1 sits in lane (16 - l) % 16 at
  // index 15 - k1 (l > 0) or in lane 0 at index 16 - k1 (l = 0, k1 > 0); the
  // second half X[8..15] of every lane is parked at S[f][lane + 16 (idx - 8)].
  const int mbase = ((16 - l) & 15) + 16 * 7 + (l == 0 ? 16 : 0);

  // Groups of 4 pairs (8 inputs, two words per sample); after a group the
  // next two words move down so that every round reads w[.][0..1].
#pragma unroll 1
  for (int g = 0; g < IN / 8; ++g) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pr = 4 * g + r;
      // Pass 1: lane n1 = l transforms z[n1 + 16 n2] over n2, z = a + i b.
      float2 x[16], X[16];
      if constexpr (TAPS == 1) {
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) {
          const uint32_t d = w[n2][r >> 1];
          if (r & 1)
            x[n2] = make_float2(sbyte<2>(d), sbyte<3>(d));
          else
            x[n2] = make_float2(sbyte<0>(d), sbyte<1>(d));
        }
      } else {
        // publish this slot's block for the pair (and, slots f < TAPS - 1,
        // block 16 + f), then sum the taps read back from P: every read of
        // the lane is at a fixed offset from one base address
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) {
          const uint32_t d = w[n2][r >> 1];
          P[f * kPRow + l + 16 * n2] = pair_f16((r & 1) ? (d >> 16) : d);
        }
        if (f < TAPS - 1) {
#pragma unroll
          for (int n2 = 0; n2 < 16; ++n2) {
            const uint32_t d = wx[n2][r >> 1];
            P[(kFBlk + f) * kPRow + l + 16 * n2] = pair_f16((r & 1) ? (d >> 16) : d);
          }
        }
        __syncthreads();
        const uint32_t* Pb = P + f * kPRow + l;
#pragma unroll
        for (int n2 = 0; n2 < 16; ++n2) {
          const float4 hv4 = hs[l + 16 * n2];
          const float hv[4] = {hv4.x, hv4.y, hv4.z, hv4.w};
          float xr = 0.f, xi = 0.f;
#pragma unroll
          for (int tp = 0; tp < TAPS; ++tp) {
            // block f + tp, sample l + 16 n2
            const half2_t q = __builtin_bit_cast(half2_t, Pb[tp * kPRow + 16 * n2]);
            xr = fmaf(hv[tp], (float)q.x, xr);
            xi = fmaf(hv[tp], (float)q.y, xi);
          }
          x[n2] = make_float2(xr, xi);
        }
      }
      dft16(x, X);
      // tw is complete (first pair); filterbank: every lane has read the
      // window before S is written
      if (TAPS > 1 || pr == 0) __syncthreads();
      S[f][l * kFSRow] = X[0];
#pragma unroll
      for (int k2 = 1; k2 < 16; ++k2) S[f][l * kFSRow + k2] = cmul(X[k2], tw[(l * k2) & (kFN - 1)]);
      wave_sync();
      // Pass 2: lane k2 = l transforms over n1; output index k = k2 + 16 k1.
#pragma unroll
      for (int n1 = 0; n1 < 16; ++n1) x[n1] = S[f][n1 * kFSRow + l];
      dft16(x, X);
      wave_sync();
#pragma unroll
      for (int k1 = 8; k1 < 16; ++k1) S[f][l + 16 * (k1 - 8)] = X[k1];
      wave_sync();
      // Split the two real inputs (X_a = (Z_k + conj Z_{N-k})/2,
      // X_b = (Z_k - conj Z_{N-k})/(2i)) and requantise channels k < 128.
      const int64_t blk_g = b0 + f;
#pragma unroll
      for (int k1 = 0; k1 < 8; ++k1) {
        const int k = l + 16 * k1;
        const float2 zk = X[k1];
        float2 zm = S[f][mbase - 16 * k1];
        if (k1 == 0 && l == 0) zm = X[0];
        const float ar = zk.x + zm.x, ai = zk.y - zm.y;
        const float br = zk.y + zm.y, bi = zm.x - zk.x;
        O[k][f] = pack4(requant_bits(ar, h, lo, hi), requant_bits(ai, h, lo, hi), requant_bits(br, h, lo, hi),
                        requant_bits(bi, h, lo, hi));
        if (a.dbg != nullptr && blk_g < a.n_blocks) {
          const int ia = i0 + 2 * pr, ib = ia + 1;
          if (ia < a.n_in)
            reinterpret_cast<float2*>(a.dbg)[((int64_t)k * a.n_in + ia) * a.n_blocks + blk_g] =
                make_float2(0.5f * ar, 0.5f * ai);
          if (ib < a.n_in)
            reinterpret_cast<float2*>(a.dbg)[((int64_t)k * a.n_in + ib) * a.n_blocks + blk_g] =
                make_float2(0.5f * br, 0.5f * bi);
        }
      }
      __syncthreads();
      // Write the pair's rows ring[k][input][t_offset + b0 ..] (32 bytes
      // each) as 16-byte pieces: piece p = tid + 256 j is half p & 1 of row
      // p >> 1 = (k, il), so two neighbouring lanes fill one row.  A piece
      // holds the il-th 16-bit half of O[k][8 half .. 8 half + 7].
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int pc = tid + 256 * j;
        const int hf = pc & 1, row = pc >> 1;
        const int k = row >> 1, il = row & 1;
        const int i = i0 + 2 * pr + il;
        if (i < a.n_in) {
          uint16_t* dst = reinterpret_cast<uint16_t*>(a.ring) + ((int64_t)k * a.n_in + i) * a.ring_stride +
                          a.t_offset + b0 + 8 * hf;
          const uint4* src = reinterpret_cast<const uint4*>(&O[k][8 * hf]);
          const uint4 q0 = src[0], q1 = src[1];
          const uint32_t sel = il ? 0x07060302u : 0x05040100u;
          const uint4 o = make_uint4(__builtin_amdgcn_perm(q0.y, q0.x, sel), __builtin_amdgcn_perm(q0.w, q0.z, sel),
                                     __builtin_amdgcn_perm(q1.y, q1.x, sel), __builtin_amdgcn_perm(q1.w, q1.z, sel));
          if (a.vec_out && nb == kFBlk) {
            *reinterpret_cast<uint4*>(dst) = o;
          } else {
            const uint32_t v[4] = {o.x, o.y, o.z, o.w};
            for (int q = 0; q < 8 && 8 * hf + q < nb; ++q) dst[q] = (uint16_t)(v[q >> 1] >> (16 * (q & 1)));
          }
        }
      }
      __syncthreads();
    }
    if constexpr (IN == 16) {
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2) {
        w[n2][0] = w[n2][2];
        w[n2][1] = w[n2][3];
      }
    }
  }
}

// 16 inputs per workgroup when n_in is a multiple of 16 (plain transform),
// else 8; the filterbank path (taps > 1, this build: 4) takes 8.
hipError_t launch_fstage(const FArgs& a, int taps, hipStream_t s) {
  if (taps != 1 && taps != 4) return hipErrorInvalidValue;
  const int in = (taps == 1 && a.n_in % 16 == 0) ? 16 : 8;
  const int64_t n_bg = (a.n_blocks + kFBlk - 1) / kFBlk;
  FArgs b = a;
  b.n_ig = (a.n_in + in - 1) / in;
  b.vec_in = (a.n_in % in == 0) && ((reinterpret_cast<uintptr_t>(a.volt) & (in - 1)) == 0);
  b.n_items = (n_bg + 3) / 4 * 4 * b.n_ig;   // block groups padded to whole ring lines
  if (b.n_items <= 0) return hipSuccess;
  b.per_xcd = (b.n_items + kNumXcd - 1) / kNumXcd;
  const int64_t grid = b.per_xcd * kNumXcd;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (taps == 4)
    hipLaunchKernelGGL((fstage_kernel<8, 4>), dim3((unsigned)grid), dim3(256), 0, s, b);
  else if (in == 16)
    hipLaunchKernelGGL((fstage_kernel<16, 1>), dim3((unsigned)grid), dim3(256), 0, s, b);
  else
    hipLaunchKernelGGL((fstage_kernel<8, 1>), dim3((unsigned)grid), dim3(256), 0, s, b);
  return hipGetLastError();
}

}  // namespace corr

namespace corr {

hipError_t launch_fstage_call(const FStageCall& c, hipStream_t s) {
  FArgs a;
  a.volt = static_cast<const int8_t*>(c.volt);
  a.twiddle = c.twiddle;
  a.ring = c.ring;
  a.dbg = c.dbg;
  a.n_blocks = c.n_blocks;
  a.ring_stride = c.ring_stride;
  a.t_offset = c.t_offset;
  a.n_in = c.n_in;
  a.scale = c.scale;
  a.max_abs = c.max_abs;
  a.vec_out = (c.t_offset % 8 == 0) && (c.ring_stride % 8 == 0) && ((reinterpret_cast<uintptr_t>(c.ring) & 15) == 0);
  a.pfb = c.pfb;
  return launch_fstage(a, c.pfb_taps > 1 ? c.pfb_taps : 1, s);
}

}  // namespace corr
