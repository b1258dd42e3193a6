// The paper's three CMAC designs (Sec. 4), kept as it describes them so that
// their ablation (Tables 2-4) can be repeated on gfx950 beside this
// library's tiled engines.  Spectra are laid out [t][input][channel]
// (channel fastest): one thread per channel, so consecutive threads read
// consecutive channels; every design accumulates all T samples in registers
// and adds into out[channel][P][2] once.
//
//   pair parallel (PP): one block per (product, 128-channel chunk); the block
//     decodes its input pair from a table in constant memory; 2 global reads
//     per product.
//   group parallel (GP, G = 2, 4): a block covers 128/G channels x G inputs of
//     a (group i, group j) pair; each thread puts its i-axis value in shared
//     memory (a barrier per sample) and reads its own j-axis value, then forms
//     G products; 2G reads per G^2 products.
//   hybrid group (HG, G = 2, 4): N_I x N_I/G blocks (the redundant half exits);
//     each thread keeps its i-axis value in shared memory (register
//     extension, no barrier) and reads G successive j-axis values; G + 1
//     reads per G products.
#include <mutex>

#include "common.h"
#include "launch.h"

namespace corr {

constexpr int kLutPairs = 128 * 129 / 2;  // products of up to 128 inputs
__constant__ uint32_t c_pair_lut[kLutPairs];  // b(i, j) = i(i+1)/2 + j -> i | j << 16

__device__ __forceinline__ void cmac(float2& acc, float2 a, float2 b) {
  // a conj(b): re = ar br + ai bi, im = ai br - ar bi
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.y, b.x, acc.y);
  acc.y = fmaf(-a.x, b.y, acc.y);
}

__device__ __forceinline__ void put(float2* out, int64_t idx, float2 v, bool diag, int accumulate) {
  if (diag) v.y = 0.f;
  if (accumulate) {
    float2 o = out[idx];
    o.x += v.x;
    o.y += v.y;
    out[idx] = o;
  } else {
    out[idx] = v;
  }
}

struct DArgs {
  const float2* x;   // [T][n_in][n_ch]
  float2* out;       // [n_ch][P]
  int64_t T;
  int64_t P;
  int32_t n_in;
  int32_t n_ch;
  int32_t accumulate;
  int32_t pad_;
};

__global__ __launch_bounds__(128) void cmac_pp_kernel(DArgs a) {
  const int c = blockIdx.x * 128 + threadIdx.x;
  const int b = blockIdx.y;
  if (c >= a.n_ch) return;
  const uint32_t ij = c_pair_lut[b];
  const int i = (int)(ij & 0xFFFFu), j = (int)(ij >> 16);
  const int64_t st = (int64_t)a.n_in * a.n_ch;
  const float2* xi = a.x + (int64_t)i * a.n_ch + c;
  const float2* xj = a.x + (int64_t)j * a.n_ch + c;
  float2 acc = make_float2(0.f, 0.f);
  for (int64_t t = 0; t < a.T; ++t) cmac(acc, xi[t * st], xj[t * st]);
  put(a.out, (int64_t)c * a.P + b, acc, i == j, a.accumulate);
}

template <int G>
__global__ __launch_bounds__(128) void cmac_gp_kernel(DArgs a) {
  constexpr int CPB = 128 / G;  // channels per block
  __shared__ float2 sa[G][CPB];
  const int cl = threadIdx.x % CPB, g = threadIdx.x / CPB;
  const int c = blockIdx.x * CPB + cl;
  const uint32_t IJ = c_pair_lut[blockIdx.y];  // group pair I >= J
  const int I = (int)(IJ & 0xFFFFu), J = (int)(IJ >> 16);
  const int ia = I * G + g, jb = J * G + g;
  const bool live = c < a.n_ch;
  const int64_t st = (int64_t)a.n_in * a.n_ch;
  const float2* xi = a.x + (int64_t)ia * a.n_ch + c;
  const float2* xj = a.x + (int64_t)jb * a.n_ch + c;
  float2 acc[G];
#pragma unroll
  for (int q = 0; q < G; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int64_t t = 0; t < a.T; ++t) {
    sa[g][cl] = live ? xi[t * st] : make_float2(0.f, 0.f);
    const float2 b = live ? xj[t * st] : make_float2(0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < G; ++q) cmac(acc[q], sa[q][cl], b);
    __syncthreads();
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int i = I * G + q;
    if (I == J && i < jb) continue;  // redundant product of a diagonal group: computed, not kept
    put(a.out, (int64_t)c * a.P + tri_index(i, jb), acc[q], i == jb, a.accumulate);
  }
}

template <int G>
__global__ __launch_bounds__(128) void cmac_hg_kernel(DArgs a) {
  __shared__ float2 sa[128];
  const int ngr = a.n_in / G;
  const int i = blockIdx.y / ngr, jg = blockIdx.y % ngr;
  if (jg * G > i) return;  // every product of this block is in the redundant half
  const int c = blockIdx.x * 128 + threadIdx.x;
  if (c >= a.n_ch) return;
  const int64_t st = (int64_t)a.n_in * a.n_ch;
  const float2* xi = a.x + (int64_t)i * a.n_ch + c;
  const float2* xj = a.x + (int64_t)(jg * G) * a.n_ch + c;
  float2 acc[G];
#pragma unroll
  for (int q = 0; q < G; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int64_t t = 0; t < a.T; ++t) {
    sa[threadIdx.x] = xi[t * st];  // this thread's own slot: no barrier needed
#pragma unroll
    for (int q = 0; q < G; ++q) cmac(acc[q], sa[threadIdx.x], xj[t * st + (int64_t)q * a.n_ch]);
  }
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const int j = jg * G + q;
    if (j > i) continue;
    put(a.out, (int64_t)c * a.P + tri_index(i, j), acc[q], i == j, a.accumulate);
  }
}

// Fill the pair table once per device (it does not depend on N_I).
static hipError_t ensure_lut() {
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (done[dev]) return hipSuccess;
  static uint32_t host[kLutPairs];
  int b = 0;
  for (int i = 0; i < 128; ++i)
    for (int j = 0; j <= i; ++j) host[b++] = (uint32_t)i | ((uint32_t)j << 16);
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_pair_lut), host, sizeof(host));
  if (e == hipSuccess) done[dev] = true;
  return e;
}

hipError_t launch_cmac_design(int design, int group, const float2* x, int64_t T, int n_in, int n_ch, float2* out,
                              int accumulate, hipStream_t s) {
  if (n_in < 1 || n_in > 128 || n_ch < 1 || T < 0) return hipErrorInvalidValue;
  DArgs a;
  a.x = x;
  a.out = out;
  a.T = T;
  a.P = (int64_t)n_in * (n_in + 1) / 2;
  a.n_in = n_in;
  a.n_ch = n_ch;
  a.accumulate = accumulate;
  a.pad_ = 0;
  hipError_t e = ensure_lut();
  if (e != hipSuccess) return e;
  if (design == 0) {
    if (group != 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(cmac_pp_kernel, dim3((unsigned)((n_ch + 127) / 128), (unsigned)a.P), dim3(128), 0, s, a);
  } else if (design == 1 || design == 2) {
    if ((group != 2 && group != 4) || n_in % group != 0) return hipErrorInvalidValue;
    const int ngr = n_in / group;
    if (design == 1) {
      const unsigned gx = (unsigned)((n_ch + 128 / group - 1) / (128 / group));
      const unsigned gy = (unsigned)(ngr * (ngr + 1) / 2);
      if (group == 2) hipLaunchKernelGGL(cmac_gp_kernel<2>, dim3(gx, gy), dim3(128), 0, s, a);
      else hipLaunchKernelGGL(cmac_gp_kernel<4>, dim3(gx, gy), dim3(128), 0, s, a);
    } else {
      const unsigned gx = (unsigned)((n_ch + 127) / 128);
      const unsigned gy = (unsigned)(n_in * ngr);
      if (group == 2) hipLaunchKernelGGL(cmac_hg_kernel<2>, dim3(gx, gy), dim3(128), 0, s, a);
      else hipLaunchKernelGGL(cmac_hg_kernel<4>, dim3(gx, gy), dim3(128), 0, s, a);
    }
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace corr
