// Device twin of synth.ci8_channel: counter-based draws of clipped rounded
// Gaussian levels, bit-identical to the numpy generator for every
// (seed, channel, input, t).  Test-signal generator only: it holds none of
// the correlator's arithmetic.
//
// Definition (both sides):
//   c   = (ch << 44) | (input << 24) | t
//   h   = mix64(mix64(seed) + c * 0x9E3779B97F4A7C15)      (SplitMix64 finaliser)
//   re  = -max_abs + #{m : lo32(h) >= thr[m]}
//   im  = -max_abs + #{m : hi32(h) >= thr[m]}
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct Thresholds {
  uint32_t t[16];
  int32_t n;
  int32_t max_abs;
};

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int level(uint32_t u, const Thresholds& th) {
  int k = -th.max_abs;
#pragma unroll
  for (int m = 0; m < 16; ++m) k += (m < th.n && u >= th.t[m]) ? 1 : 0;
  return k;
}

// One thread writes 8 consecutive samples (16 bytes) of one (channel, input) row.
__global__ void fill_ci8_kernel(int8_t* __restrict__ out, int64_t ch0, int64_t n_in,
                                int64_t n_t, int64_t row_stride, int64_t n_rows,
                                uint64_t key, Thresholds th) {
  const int64_t groups_per_row = (n_t + 7) / 8;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_rows * groups_per_row) return;
  const int64_t row = gid / groups_per_row;
  const int64_t t0 = (gid - row * groups_per_row) * 8;
  const uint64_t ch = (uint64_t)(ch0 + row / n_in);
  const uint64_t inp = (uint64_t)(row % n_in);
  const uint64_t base = (ch << 44) | (inp << 24);
  int8_t* dst = out + (row * row_stride + t0) * 2;
  int8_t v[16];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    const uint64_t h = mix64(key + (base | (uint64_t)(t0 + s)) * 0x9E3779B97F4A7C15ull);
    v[2 * s] = (int8_t)level((uint32_t)h, th);
    v[2 * s + 1] = (int8_t)level((uint32_t)(h >> 32), th);
  }
  if (t0 + 8 <= n_t && ((reinterpret_cast<uintptr_t>(dst) & 15) == 0)) {
    *reinterpret_cast<int4*>(dst) = *reinterpret_cast<const int4*>(v);
  } else {
    for (int s = 0; s < 8 && t0 + s < n_t; ++s) {
      dst[2 * s] = v[2 * s];
      dst[2 * s + 1] = v[2 * s + 1];
    }
  }
}

uint64_t host_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

// Fill int8 pairs [n_ch][n_in][row_stride][2] for channels ch0..ch0+n_ch-1 and
// samples 0..n_t-1 of each row.  Returns 0 on success, -1 on bad arguments,
// -3 on a HIP launch error.  Asynchronous on `stream`.
extern "C" int synth_fill_ci8(void* d_out, int64_t ch0, int64_t n_ch, int64_t n_in, int64_t n_t,
                              int64_t row_stride, uint64_t seed, const Thresholds* th,
                              void* stream) {
  if (!d_out || !th || n_ch < 0 || n_in < 0 || n_t < 0 || row_stride < n_t || ch0 < 0) return -1;
  if (th->n < 0 || th->n > 16) return -1;
  if (ch0 + n_ch > (1ll << 20) || n_in > (1ll << 20) || n_t > (1ll << 24)) return -1;
  const int64_t rows = n_ch * n_in;
  const int64_t work = rows * ((n_t + 7) / 8);
  if (work == 0) return 0;
  const int block = 256;
  const int64_t grid = (work + block - 1) / block;
  if (grid > 0x7FFFFFFF) return -1;
  hipLaunchKernelGGL(fill_ci8_kernel, dim3((unsigned)grid), dim3(block), 0, (hipStream_t)stream,
                     (int8_t*)d_out, ch0, n_in, n_t, row_stride, rows, host_mix64(seed), *th);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

namespace {
struct JobFill {
  uint64_t base_seed;
  Thresholds th;
};
}  // namespace

// Fill callback for the serving scheduler: job `job_id` gets the ci8 signal
// of seed base_seed + job_id in rows of row_stride samples (user points to a
// JobFill).  Queues one kernel on
// `stream`; never blocks.
extern "C" void synth_fill_job(void* user, uint64_t job_id, void* d_samples, int64_t n_ch, int64_t n_in,
                               int64_t n_t, int64_t row_stride, void* stream) {
  const JobFill* f = static_cast<const JobFill*>(user);
  synth_fill_ci8(d_samples, 0, n_ch, n_in, n_t, row_stride, f->base_seed + job_id, &f->th, stream);
}
