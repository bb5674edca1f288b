// Device helpers shared by the library's kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace spamm {

constexpr int kWave = 64;

// Pointers read from descriptor tables lose their address space, and the
// compiler then emits flat loads, which also count against lgkmcnt: every
// wait on an LDS read would then wait for outstanding global loads too.
// These casts restore the global address space (and scalar loads where the
// address is wave-uniform).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}

// Morton (Z-order) key of block (r, c): row bit above column bit, so the
// four children of node m are 4m + 2a + b for (2r + a, 2c + b).
__device__ __forceinline__ uint32_t spread_bits(uint32_t x) {
  x &= 0x0000ffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}
__device__ __forceinline__ uint32_t compact_bits(uint32_t x) {
  x &= 0x55555555u;
  x = (x | (x >> 1)) & 0x33333333u;
  x = (x | (x >> 2)) & 0x0f0f0f0fu;
  x = (x | (x >> 4)) & 0x00ff00ffu;
  x = (x | (x >> 8)) & 0x0000ffffu;
  return x;
}
__device__ __forceinline__ uint32_t morton(uint32_t r, uint32_t c) {
  return (spread_bits(r) << 1) | spread_bits(c);
}
__device__ __forceinline__ void demorton(uint32_t m, uint32_t& r, uint32_t& c) {
  r = compact_bits(m >> 1);
  c = compact_bits(m);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Tree sum over the 64 lanes; every lane returns lane 0's value, so the
// association order is fixed and the result is bitwise reproducible.
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, kWave);
  return __shfl(v, 0, kWave);
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, kWave);
  return __shfl(v, 0, kWave);
}
__device__ __forceinline__ int wave_or_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v |= __shfl_down(v, off, kWave);
  return __shfl(v, 0, kWave);
}

// Block sum: per-wave tree sums combined by wave 0 in wave order.  `red`
// must hold blockDim/64 doubles.  Returns the sum in every thread.
__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  v = wave_sum_f64(v);
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }
__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

}  // namespace spamm
