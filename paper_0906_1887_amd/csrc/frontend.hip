// Complex front end of the prototype correlator.
//
// Aggregation (Sec. 3): every capture stream is a run of records of one
// marker/counter word and one 16-bit word per receiver input; the aggregator
// drops the marker words and interleaves the streams so that all inputs of
// one time instant are adjacent.  The marker is taken as a 16-bit record
// counter, and records whose counter is not the expected one in some stream
// are counted (the data are copied regardless).
//
// Complex F-stage (Sec. 2, Sec. 4): for complex samples N_C samples give N_C
// channels.  Input formats: 5-bit real and imaginary parts in two's
// complement in a 16-bit word (Sec. 3; re = bits 9..5, im = bits 4..0), or
// the 1-byte mode with one bit less of each (Sec. 5; re = bits 7..4,
// im = bits 3..0).  The unpack is fused into the load; each 128-sample block
// of each input is transformed by a 128-point complex FFT (16 x 8 four-step:
// 8 lanes per FFT, a DFT16 per lane, the inner twiddles, one wave-local LDS
// exchange, two DFT8s per lane), requantised like the real F-stage and
// written to ring[k][input][t] for k = 0..127 in natural order (DC first).
#include "common.h"
#include "fft_device.h"
#include "launch.h"

namespace corr {

// --------------------------------------------------------------- aggregation

// One thread per output word: out[r][s * w_per + w] = rec[s][r][1 + w].
// The thread of word 0 of row r checks the counters of record r.
__global__ __launch_bounds__(256) void aggregate_w16_kernel(const uint16_t* __restrict__ rec, int32_t n_streams,
                                                            int32_t w_per, int64_t n_rec, uint32_t first_counter,
                                                            uint16_t* __restrict__ out, uint32_t* __restrict__ bad) {
  const int64_t row = (int64_t)n_streams * w_per;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= n_rec * row) return;
  const int64_t r = t / row;
  const int32_t j = (int32_t)(t - r * row);
  const int32_t s = j / w_per, w = j - s * w_per;
  const int64_t rec_words = 1 + (int64_t)w_per;
  out[t] = rec[((int64_t)s * n_rec + r) * rec_words + 1 + w];
  if (j == 0 && bad != nullptr) {
    const uint16_t want = (uint16_t)((first_counter + (uint64_t)r) & 0xFFFFu);
    bool mismatch = false;
    for (int32_t q = 0; q < n_streams; ++q) mismatch |= (rec[((int64_t)q * n_rec + r) * rec_words] != want);
    if (mismatch) atomicAdd(bad, 1u);
  }
}

// The prototype's layout (16 words per record, up to 4 streams): a workgroup
// copies 128 records of every stream into LDS (128 records x 34 bytes is a
// whole number of 16-byte pieces; VEC loads 16 bytes per lane and needs every
// stream's run 16-byte aligned, else dwords), then writes its output rows as
// one contiguous run of 16-byte pieces and checks the counters.  Each piece
// is five LDS dwords funnel-shifted by 0 or 16 bits, since a record's samples
// start 2 bytes past its marker.  At 17.5 KB of LDS, eight workgroups fit
// on a CU.
constexpr int kAggRec = 128;
constexpr int kAggWords = 17;                          // marker + 16 samples
constexpr int kAggDw = kAggRec * kAggWords / 2;        // dwords per stream
constexpr int kAggPitch = kAggDw + 8;                  // streams 8 banks apart
static_assert(kAggDw % 4 == 0 && kAggPitch % 4 == 0, "16-byte LDS rows");
template <bool VEC>
__global__ __launch_bounds__(256) void aggregate_w16_rows_kernel(const uint16_t* __restrict__ rec, int32_t n_streams,
                                                                 int64_t n_rec, uint32_t first_counter,
                                                                 uint16_t* __restrict__ out,
                                                                 uint32_t* __restrict__ bad) {
  __shared__ __align__(16) uint32_t buf[4 * kAggPitch];  // 17.5 KB; kAggPitch is a multiple of 4
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kAggRec;
  const int nr = (int)min((int64_t)kAggRec, n_rec - r0);  // even: n_rec and r0 are
  const int nd = nr * kAggWords / 2;
  // One flat loop over every stream's run keeps all lanes loading.
  if (VEC) {
    const int nq = nd / 4;   // nr is a multiple of 8 here, so nd is a multiple of 4
    for (int d = tid; d < n_streams * nq; d += 256) {
      const int s = d / nq, q = d - s * nq;
      const uint4* src4 = reinterpret_cast<const uint4*>(rec + ((int64_t)s * n_rec + r0) * kAggWords);
      reinterpret_cast<uint4*>(buf + s * kAggPitch)[q] = src4[q];
    }
  } else {
    for (int d = tid; d < n_streams * nd; d += 256) {
      const int s = d / nd, q = d - s * nd;
      const uint32_t* src = reinterpret_cast<const uint32_t*>(rec + ((int64_t)s * n_rec + r0) * kAggWords);
      buf[s * kAggPitch + q] = src[q];
    }
  }
  __syncthreads();
  // Output: the workgroup's rows are one contiguous run of nr * n_streams * 32
  // bytes; 16-byte piece p holds half (p % 2) of stream (p / 2 % n_streams)'s
  // samples of record p / (2 n_streams), so each store instruction writes
  // 1 KB in one run.
  const int pieces = nr * n_streams * 2;
  uint4* dst = reinterpret_cast<uint4*>(out + r0 * (int64_t)n_streams * 16);
  for (int pc = tid; pc < pieces; pc += 256) {
    const int r = pc / (2 * n_streams);
    const int s = (pc >> 1) - r * n_streams;
    const int o = r * (2 * kAggWords) + 2 + 16 * (pc & 1);   // byte offset of the piece in its stream
    const uint32_t* b = buf + s * kAggPitch + (o >> 2);
    const uint32_t sh = (uint32_t)(o & 3) * 8;                 // 0 or 16
    uint32_t w[5];
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = b[q];
    w[4] = sh ? b[4] : 0u;                                     // b[4] lies inside the record when sh != 0
    dst[pc] = make_uint4(__builtin_amdgcn_alignbit(w[1], w[0], sh), __builtin_amdgcn_alignbit(w[2], w[1], sh),
                         __builtin_amdgcn_alignbit(w[3], w[2], sh), __builtin_amdgcn_alignbit(w[4], w[3], sh));
  }
  // Counters: thread r checks record r of every stream.
  if (tid >= nr) return;
  const uint16_t want = (uint16_t)((first_counter + (uint64_t)(r0 + tid)) & 0xFFFFu);
  bool mismatch = false;
  for (int s = 0; s < n_streams; ++s)
    mismatch |= (reinterpret_cast<const uint16_t*>(buf + s * kAggPitch)[tid * kAggWords] != want);
  if (mismatch && bad != nullptr) atomicAdd(bad, 1u);
}

hipError_t launch_aggregate_w16(const uint16_t* rec, int32_t n_streams, int32_t w_per, int64_t n_rec,
                                uint32_t first_counter, uint16_t* out, uint32_t* bad, hipStream_t s) {
  const int64_t total = n_rec * n_streams * (int64_t)w_per;
  if (total <= 0) return hipSuccess;
  if (w_per == 16 && n_streams <= 4 && n_rec % 2 == 0 && (reinterpret_cast<uintptr_t>(rec) & 3) == 0 &&
      (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
    const int64_t grid = (n_rec + kAggRec - 1) / kAggRec;
    if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
    // 16-byte loads: every stream's run of kAggRec records starts 16-byte aligned.
    const bool vec = (reinterpret_cast<uintptr_t>(rec) & 15) == 0 && n_rec % 8 == 0;
    if (vec)
      hipLaunchKernelGGL(aggregate_w16_rows_kernel<true>, dim3((unsigned)grid), dim3(256), 0, s, rec, n_streams,
                         n_rec, first_counter, out, bad);
    else
      hipLaunchKernelGGL(aggregate_w16_rows_kernel<false>, dim3((unsigned)grid), dim3(256), 0, s, rec, n_streams,
                         n_rec, first_counter, out, bad);
    return hipGetLastError();
  }
  const int64_t grid = (total + 255) / 256;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(aggregate_w16_kernel, dim3((unsigned)grid), dim3(256), 0, s, rec, n_streams, w_per, n_rec,
                     first_counter, out, bad);
  return hipGetLastError();
}

// --------------------------------------------------------- complex F-stage

constexpr int kCN = 128;     // FFT length = channels
constexpr int kCBlk = 16;    // blocks per workgroup
constexpr int kCSlots = 32;  // FFT slots of 8 lanes
constexpr int kCSRow = 17;   // padded row (16 entries) of the 8 x 16 exchange
constexpr int kCORow = 20;   // words per channel row of O (16 blocks + pad, 16-byte aligned rows)

struct CArgs {
  const uint8_t* volt;     // [n_blocks*128][n_in] samples of SB bytes
  const float2* twiddle;   // W_128^m, m = 0..127
  int8_t* ring;            // [128][n_in][ring_stride][2]
  float* dbg;              // optional [128][n_in][n_blocks][2]
  int64_t n_blocks;
  int64_t ring_stride;
  int64_t t_offset;
  int32_t n_in;
  int32_t n_ig;            // ceil(n_in / inputs per workgroup)
  float scale;
  float max_abs;
  int32_t vec_in;          // n_in a multiple of the inputs per workgroup, volt 16-byte aligned
  int32_t vec_out;         // t_offset, ring_stride multiples of 8, ring 16-byte aligned
  int64_t n_items;
  int64_t per_xcd;
};

// Sample (re, im) of input j (0..IN-1) from the 16 bytes a lane holds for
// one time instant.  FMT 1: 16-bit words, 5+5 bits; FMT 2: bytes, 4+4 bits.
template <int FMT>
__device__ __forceinline__ float2 unpack_sample(uint32_t d, int shift) {
  const uint32_t v = d >> shift;
  if constexpr (FMT == 1)
    return make_float2((float)((int32_t)(v << 22) >> 27), (float)((int32_t)(v << 27) >> 27));
  else
    return make_float2((float)((int32_t)(v << 24) >> 28), (float)((int32_t)(v << 28) >> 28));
}

// One workgroup: 16 blocks x 8 inputs (16 bytes per time instant for 16-bit
// words, 8 for bytes).  Slot f = tid / 8 (lanes l = tid % 8) owns block
// f % 16 and, in round pr, input 2 pr + f / 16 (the two inputs of a round sit
// in different waves); it loads its 16 samples x 8 inputs straight into
// registers.  S[f] is used by the 8 lanes of slot f only, all in one wave; O
// is the workgroup's corner turn for the round.
template <int FMT>
__global__ __launch_bounds__(256, 3) void fstage_c_kernel(CArgs a) {
  constexpr int SB = (FMT == 1) ? 2 : 1;  // bytes per sample
  constexpr int IN = 8;                   // inputs per workgroup
  constexpr int NW = 2 * SB;              // 32-bit words per time instant and lane
  __shared__ __attribute__((aligned(16))) float2 S[kCSlots][8 * kCSRow];  // 34 KB
  __shared__ __attribute__((aligned(16))) uint32_t O[kCN][kCORow];         // 10 KB
  __shared__ float2 tw[kCN];                                               // 1 KB

  const int tid = threadIdx.x;
  const int64_t item = xcd_item(blockIdx.x, a.per_xcd);
  if ((int64_t)(blockIdx.x / kNumXcd) >= a.per_xcd || item >= a.n_items) return;
  // Items run through 4 consecutive block groups of one input group (the
  // four 32-byte pieces of each 128-byte ring line), then input groups, then
  // the next 4 block groups.
  const int64_t rest = item >> 2;
  const int ig = (int)(rest % a.n_ig);
  const int64_t b0 = ((rest / a.n_ig) * 4 + (item & 3)) * kCBlk;
  if (b0 >= a.n_blocks) return;
  const int i0 = ig * IN;
  const int f = tid >> 3;
  const int l = tid & 7;
  const int blk = f & (kCBlk - 1);
  const int hi = f >> 4;  // which input of the round's pair (uniform per wave)
  const int64_t nb = min((int64_t)kCBlk, a.n_blocks - b0);

  // Samples t = l + 8 n2 of block b0 + blk, inputs i0..i0+IN-1 (zero outside).
  uint32_t w[16][NW];
  if (a.vec_in && nb == kCBlk) {
    const uint8_t* p = a.volt + (((b0 + blk) * kCN + l) * a.n_in + i0) * SB;
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) {
      const uint8_t* q = p + (int64_t)n2 * 8 * a.n_in * SB;
      if constexpr (NW == 4) {
        const uint4 v = *reinterpret_cast<const uint4*>(q);
        w[n2][0] = v.x; w[n2][1] = v.y; w[n2][2] = v.z; w[n2][3] = v.w;
      } else {
        const uint2 v = *reinterpret_cast<const uint2*>(q);
        w[n2][0] = v.x; w[n2][1] = v.y;
      }
    }
  } else {
#pragma unroll
    for (int n2 = 0; n2 < 16; ++n2) {
      const int64_t t = (b0 + blk) * kCN + l + 8 * n2;
      const uint8_t* p = a.volt + (t * a.n_in + i0) * SB;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        uint32_t v = 0;
        for (int q = 0; q < 4; ++q) {
          const int byte = 4 * j + q;
          if (blk < nb && i0 + byte / SB < a.n_in) v |= (uint32_t)p[byte] << (8 * q);
        }
        w[n2][j] = v;
      }
    }
  }
  if (tid < kCN) tw[tid] = a.twiddle[tid];

  const float h = a.scale;
  const float lo = kRqMagic - a.max_abs, hi_b = kRqMagic + a.max_abs;

  // One round per input pair.  This slot's sample of round pr sits in word 0
  // at bit 16 hi (16-bit words) or 8 hi (bytes); after a round the next pair
  // is brought there (words move down; for bytes, every other round shifts
  // word 0 down by 16 bits instead).  Fully unrolled, those moves become
  // register renames.
  const int shift = (FMT == 1) ? 16 * hi : 8 * hi;
#pragma unroll
  for (int pr = 0; pr < IN / 2; ++pr) {
    {
      float2 x[16], X[16];
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2) x[n2] = unpack_sample<FMT>(w[n2][0], shift);
      // Pass 1: lane n1 = l transforms x[n1 + 8 n2] over n2; inner twiddle W_128^(n1 k2).
      dft16(x, X);
      if (pr == 0) __syncthreads();  // tw is complete
      S[f][l * kCSRow] = X[0];
#pragma unroll
      for (int k2 = 1; k2 < 16; ++k2) S[f][l * kCSRow + k2] = cmul(X[k2], tw[(l * k2) & (kCN - 1)]);
      wave_sync();
      // Pass 2: DFT8 over n1 for k2 = l and then k2 = l + 8; output
      // k = k2 + 16 k1, requantised into O (the 16-bit half of this slot's
      // input).
      const int i = i0 + 2 * pr + hi;
      const int64_t blk_g = b0 + blk;
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        float2 y[8], z[8];
#pragma unroll
        for (int n1 = 0; n1 < 8; ++n1) y[n1] = S[f][n1 * kCSRow + l + 8 * h2];
        dft8(y, z);
#pragma unroll
        for (int k1 = 0; k1 < 8; ++k1) {
          const int k = l + 8 * h2 + 16 * k1;
          const uint32_t code = __builtin_amdgcn_perm(requant_bits(z[k1].y, h, lo, hi_b),
                                                      requant_bits(z[k1].x, h, lo, hi_b), 0x0c0c0400u);
          reinterpret_cast<uint16_t*>(&O[k][blk])[hi] = (uint16_t)code;
          if (a.dbg != nullptr && blk_g < a.n_blocks && i < a.n_in)
            reinterpret_cast<float2*>(a.dbg)[((int64_t)k * a.n_in + i) * a.n_blocks + blk_g] = z[k1];
        }
      }
      __syncthreads();
      // Write the pair's rows ring[k][input][t_offset + b0 ..] (32 bytes
      // each) as 16-byte pieces, two neighbouring lanes per row; a piece
      // holds the il-th 16-bit half of O[k][8 half .. 8 half + 7].
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int pc = tid + 256 * j;
        const int hf = pc & 1, row = pc >> 1;
        const int k = row >> 1, il = row & 1;
        const int io = i0 + 2 * pr + il;
        if (io < a.n_in) {
          uint16_t* dst = reinterpret_cast<uint16_t*>(a.ring) + ((int64_t)k * a.n_in + io) * a.ring_stride +
                          a.t_offset + b0 + 8 * hf;
          const uint4* src = reinterpret_cast<const uint4*>(&O[k][8 * hf]);
          const uint4 q0 = src[0], q1 = src[1];
          const uint32_t sel = il ? 0x07060302u : 0x05040100u;
          const uint4 o = make_uint4(__builtin_amdgcn_perm(q0.y, q0.x, sel), __builtin_amdgcn_perm(q0.w, q0.z, sel),
                                     __builtin_amdgcn_perm(q1.y, q1.x, sel), __builtin_amdgcn_perm(q1.w, q1.z, sel));
          if (a.vec_out && nb == kCBlk) {
            *reinterpret_cast<uint4*>(dst) = o;
          } else {
            const uint32_t v[4] = {o.x, o.y, o.z, o.w};
            for (int q = 0; q < 8 && 8 * hf + q < nb; ++q) dst[q] = (uint16_t)(v[q >> 1] >> (16 * (q & 1)));
          }
        }
      }
      __syncthreads();
    }
    if (FMT == 2 && (pr & 1) == 0) {
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2) w[n2][0] >>= 16;
    } else {
#pragma unroll
      for (int n2 = 0; n2 < 16; ++n2)
#pragma unroll
        for (int j = 0; j + 1 < NW; ++j) w[n2][j] = w[n2][j + 1];
    }
  }
}

hipError_t launch_fstage_complex(const FStageCall& c, hipStream_t s) {
  if (c.format != 1 && c.format != 2) return hipErrorInvalidValue;
  const int sb = (c.format == 1) ? 2 : 1;
  const int in = 8;
  CArgs a;
  a.volt = reinterpret_cast<const uint8_t*>(c.volt);
  a.twiddle = c.twiddle;
  a.ring = c.ring;
  a.dbg = c.dbg;
  a.n_blocks = c.n_blocks;
  a.ring_stride = c.ring_stride;
  a.t_offset = c.t_offset;
  a.n_in = c.n_in;
  a.n_ig = (c.n_in + in - 1) / in;
  a.scale = c.scale;
  a.max_abs = c.max_abs;
  a.vec_in = (c.n_in % in == 0) && ((reinterpret_cast<uintptr_t>(c.volt) & (in * sb - 1)) == 0);
  a.vec_out = (c.t_offset % 8 == 0) && (c.ring_stride % 8 == 0) && ((reinterpret_cast<uintptr_t>(c.ring) & 15) == 0);
  const int64_t n_bg = (c.n_blocks + kCBlk - 1) / kCBlk;
  a.n_items = (n_bg + 3) / 4 * 4 * a.n_ig;   // block groups padded to whole lines
  if (a.n_items <= 0) return hipSuccess;
  a.per_xcd = (a.n_items + kNumXcd - 1) / kNumXcd;
  const int64_t grid = a.per_xcd * kNumXcd;
  if (grid > 0x7FFFFFFF) return hipErrorInvalidValue;
  if (c.format == 1)
    hipLaunchKernelGGL(fstage_c_kernel<1>, dim3((unsigned)grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(fstage_c_kernel<2>, dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace corr
