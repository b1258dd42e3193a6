// Accumulator maintenance: ordered reduction of K-split partial tiles into the
// integration accumulator, the FP64 long-run fold, and fills.
//
// Fig. 1: the accumulators are read after an interval, divided by the number
// of updates (left to the caller, who gets the raw sums and the count) and
// reset.  The long-run fold keeps L += V in FP64 across many integrations.
#include "common.h"
#include "launch.h"

namespace corr {

// acc[k] = (accumulate ? acc[k] : 0) + part[0][k] + part[1][k] + ... in that
// order (integer sums are exact; the fixed order keeps float sums
// reproducible).  n = number of (re, im) pairs per partial buffer.  A thread
// takes two neighbouring pairs (wide: one 16-byte load per split, when n is
// even and both buffers are 16-byte aligned) and issues the loads of four
// splits before adding them in split order, so several loads are in flight
// per thread.
template <typename T2>
struct Wide;
template <>
struct Wide<int2> { typedef int4 T; };
template <>
struct Wide<float2> { typedef float4 T; };

template <typename T4>
__device__ __forceinline__ void add4(T4& s, const T4& p) {
  s.x += p.x;
  s.y += p.y;
  s.z += p.z;
  s.w += p.w;
}

template <typename T2>
__global__ void reduce_splits_kernel(const T2* __restrict__ part, int64_t n, int n_split,
                                     T2* __restrict__ acc, int accumulate, int wide) {
  using T4 = typename Wide<T2>::T;
  const int64_t k = 2 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);   // first pair
  if (k >= n) return;
  if (wide) {
    const T4* __restrict__ p4 = reinterpret_cast<const T4*>(part);
    const int64_t n4 = n / 2, k4 = k / 2;
    T4 s = p4[k4];
    int q = 1;
    for (; q + 3 < n_split; q += 4) {
      const T4 a = p4[(int64_t)q * n4 + k4], b = p4[(int64_t)(q + 1) * n4 + k4];
      const T4 c = p4[(int64_t)(q + 2) * n4 + k4], d = p4[(int64_t)(q + 3) * n4 + k4];
      add4(s, a);
      add4(s, b);
      add4(s, c);
      add4(s, d);
    }
    for (; q < n_split; ++q) add4(s, p4[(int64_t)q * n4 + k4]);
    T4* __restrict__ a4 = reinterpret_cast<T4*>(acc);
    if (accumulate) {
      T4 o = a4[k4];
      add4(o, s);   // o + s: the same operand order as the pair path below
      s = o;
    }
    a4[k4] = s;
    return;
  }
  for (int64_t kk = k; kk < min(k + 2, n); ++kk) {   // pair by pair
    T2 s = part[kk];
    for (int q = 1; q < n_split; ++q) {
      const T2 p = part[(int64_t)q * n + kk];
      s.x += p.x;
      s.y += p.y;
    }
    if (accumulate) {
      const T2 o = acc[kk];
      s.x = o.x + s.x;
      s.y = o.y + s.y;
    }
    acc[kk] = s;
  }
}

// L[k] += (double) V[k] over n scalars (the (re, im) pairs flattened).
template <typename T>
__global__ void fold_f64_kernel(double* __restrict__ L, const T* __restrict__ V, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) L[k] += (double)V[k];
}

__global__ void fill_zero_kernel(uint4* __restrict__ p, int64_t n16) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n16) p[k] = make_uint4(0u, 0u, 0u, 0u);
}

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

hipError_t launch_reduce_splits(const void* part, int64_t n_pairs, int n_split, void* acc, int accumulate,
                                bool is_int, hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  // two pairs per thread
  const int64_t threads = (n_pairs + 1) / 2;
  const int wide = (n_pairs % 2 == 0) && (((reinterpret_cast<uintptr_t>(part) | reinterpret_cast<uintptr_t>(acc)) & 15) == 0);
  if (is_int)
    hipLaunchKernelGGL(reduce_splits_kernel<int2>, dim3(grid_for(threads, 256)), dim3(256), 0, s,
                       static_cast<const int2*>(part), n_pairs, n_split, static_cast<int2*>(acc), accumulate, wide);
  else
    hipLaunchKernelGGL(reduce_splits_kernel<float2>, dim3(grid_for(threads, 256)), dim3(256), 0, s,
                       static_cast<const float2*>(part), n_pairs, n_split, static_cast<float2*>(acc), accumulate,
                       wide);
  return hipGetLastError();
}

hipError_t launch_fold_f64(double* L, const void* V, int64_t n_scalars, bool is_int, hipStream_t s) {
  if (n_scalars <= 0) return hipSuccess;
  if (is_int)
    hipLaunchKernelGGL(fold_f64_kernel<int32_t>, dim3(grid_for(n_scalars, 256)), dim3(256), 0, s, L,
                       static_cast<const int32_t*>(V), n_scalars);
  else
    hipLaunchKernelGGL(fold_f64_kernel<float>, dim3(grid_for(n_scalars, 256)), dim3(256), 0, s, L,
                       static_cast<const float*>(V), n_scalars);
  return hipGetLastError();
}

// Zero `bytes` (a multiple of 16) at a 16-byte aligned device pointer.
hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s) {
  const int64_t n16 = bytes / 16;
  if (n16 <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(n16, 256)), dim3(256), 0, s, static_cast<uint4*>(p), n16);
  return hipGetLastError();
}

// Any address and length (a kernel, not a memset node, also under stream capture).
__global__ void fill_zero_bytes_kernel(uint8_t* __restrict__ p, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) p[k] = 0;
}

hipError_t launch_fill_zero_bytes(void* p, int64_t bytes, hipStream_t s) {
  if (bytes <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_bytes_kernel, dim3(grid_for(bytes, 256)), dim3(256), 0, s, static_cast<uint8_t*>(p),
                     bytes);
  return hipGetLastError();
}

// Guard word w of band g: a position-dependent pattern, so that a band copied
// or shifted onto another is also seen.
__device__ __forceinline__ uint32_t guard_word(int g, int w) {
  return 0xA5C3F00Du ^ ((uint32_t)(g * (kGuardBytes / 4) + w) * 0x9E3779B1u);
}

__global__ void guard_fill_kernel(uint8_t* __restrict__ ws, GuardList gl) {
  const int g = blockIdx.x, w = threadIdx.x;   // one block per band, one thread per word
  reinterpret_cast<uint32_t*>(ws + gl.off[g])[w] = guard_word(g, w);
}

// One workgroup: count the band words that differ from the pattern.
__global__ void guard_check_kernel(const uint8_t* __restrict__ ws, GuardList gl, uint32_t* __restrict__ bad) {
  __shared__ uint32_t count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  constexpr int kWords = kGuardBytes / 4;
  uint32_t n = 0;
  for (int k = threadIdx.x; k < gl.n * kWords; k += blockDim.x) {
    const int g = k / kWords, w = k % kWords;
    n += reinterpret_cast<const uint32_t*>(ws + gl.off[g])[w] != guard_word(g, w) ? 1u : 0u;
  }
  if (n) atomicAdd(&count, n);
  __syncthreads();
  if (threadIdx.x == 0) *bad = count;
}

hipError_t launch_guard_fill(uint8_t* ws, const GuardList& g, hipStream_t s) {
  if (g.n <= 0) return hipSuccess;
  if (g.n > kMaxGuards) return hipErrorInvalidValue;
  hipLaunchKernelGGL(guard_fill_kernel, dim3(g.n), dim3(kGuardBytes / 4), 0, s, ws, g);
  return hipGetLastError();
}

hipError_t launch_guard_check(const uint8_t* ws, const GuardList& g, uint32_t* bad, hipStream_t s) {
  if (g.n > kMaxGuards) return hipErrorInvalidValue;
  hipLaunchKernelGGL(guard_check_kernel, dim3(1), dim3(256), 0, s, ws, g, bad);
  return hipGetLastError();
}

}  // namespace corr
