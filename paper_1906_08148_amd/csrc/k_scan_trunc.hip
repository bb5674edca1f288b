// LDS-staged exclusive prefix scans, and input truncation with a global
// Frobenius budget (leaf-block form of Sec. 3's vector-space truncation).
#include "internal.h"
#include "kern_common.h"

namespace spamm {

constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

// ---------------------------------------------------------------- scan

template <typename In>
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const In* __restrict__ in, int64_t count,
                                                            int64_t* __restrict__ sums) {
  __shared__ int64_t red[kScanThreads / kWave];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  int64_t v = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + int64_t(i) * kScanThreads + threadIdx.x;
    if (idx < count) v += int64_t(in[idx]);
  }
  v = wave_sum_i64(v);
  if (lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
    sums[blockIdx.x] = t;
  }
}

// Inclusive scan over the 64 lanes.
__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int64_t t = __shfl_up(v, off, kWave);
    if (l >= off) v += t;
  }
  return v;
}

// Exclusive scan of the tile sums by one workgroup, carrying across chunks.
__global__ void __launch_bounds__(1024) k_scan_top(int64_t* __restrict__ sums, int64_t nb,
                                                   int64_t* __restrict__ total) {
  __shared__ int64_t wtot[1024 / kWave];
  __shared__ int64_t carry_sh;
  if (threadIdx.x == 0) carry_sh = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t idx = base + threadIdx.x;
    const int64_t v = idx < nb ? sums[idx] : 0;
    const int64_t inc = wave_incl_scan(v);
    if (lane_id() == kWave - 1) wtot[threadIdx.x / kWave] = inc;
    __syncthreads();
    int64_t wpre = 0;
    for (int w = 0; w < int(threadIdx.x / kWave); ++w) wpre += wtot[w];
    const int64_t carry = carry_sh;
    if (idx < nb) sums[idx] = carry + wpre + inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry_sh = carry + wpre + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry_sh;
}

// mode 0: out64[i] = exclusive prefix; mode 1: out32[i] = in[i] ? prefix : -1
template <typename In, int Mode>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const In* __restrict__ in, int64_t count,
                                                            const int64_t* __restrict__ offs,
                                                            int64_t* __restrict__ out64,
                                                            int32_t* __restrict__ out32) {
  __shared__ int64_t wtot[kScanThreads / kWave];
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int64_t vals[kScanItems];
  int64_t local = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    vals[i] = idx < count ? int64_t(in[idx]) : 0;
    local += vals[i];
  }
  const int64_t inc = wave_incl_scan(local);
  if (lane_id() == kWave - 1) wtot[threadIdx.x / kWave] = inc;
  __syncthreads();
  int64_t run = offs[blockIdx.x] + inc - local;
  for (int w = 0; w < int(threadIdx.x / kWave); ++w) run += wtot[w];
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < count) {
      if (Mode == 0) out64[idx] = run;
      else out32[idx] = vals[i] ? int32_t(run) : -1;
    }
    run += vals[i];
  }
}

size_t scan_scratch_bytes(int64_t count) {
  const int64_t nb = (count + kScanTile - 1) / kScanTile;
  return size_t((nb + 1) * sizeof(int64_t) + 256);
}

template <typename In, int Mode>
static hipError_t scan_impl(hipStream_t s, const In* in, int64_t count, int64_t* out64, int32_t* out32,
                            int64_t* total, void* scratch, size_t scratch_bytes) {
  const int64_t nb = std::max<int64_t>(1, (count + kScanTile - 1) / kScanTile);
  if (scratch_bytes < size_t(nb * sizeof(int64_t))) return hipErrorInvalidValue;
  int64_t* sums = static_cast<int64_t*>(scratch);
  hipLaunchKernelGGL((k_scan_tiles<In>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, s, in, count, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, sums, nb, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_scan_apply<In, Mode>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, s, in, count,
                     sums, out64, out32);
  return hipGetLastError();
}

hipError_t launch_scan_i64(hipStream_t s, const int64_t* in, int64_t* out, int64_t count, void* scratch,
                           size_t scratch_bytes) {
  return scan_impl<int64_t, 0>(s, in, count, out, nullptr, out + count, scratch, scratch_bytes);
}

hipError_t launch_flags_to_slots(hipStream_t s, const int32_t* flag, int64_t count, int32_t* slot,
                                 int64_t* total, void* scratch, size_t scratch_bytes) {
  return scan_impl<int32_t, 1>(s, flag, count, nullptr, slot, total, scratch, scratch_bytes);
}

// ---------------------------------------------------------------- truncation
//
// Order the non-null leaves by the key (bits of the squared norm s, Morton
// index m) -- for s >= 0 the IEEE bit pattern orders like the value -- and
// drop the longest prefix whose summed squared norm is <= tau^2.  Only leaves
// with s <= tau^2 can be in that prefix.  Instead of sorting, the largest key
// K with F(K) = sum{ s : key <= K } <= tau^2 is built bit by bit from the top;
// F is evaluated in one fixed order (a thread's strided share, then a fixed
// tree), so each addition only grows with K and F is monotone in K.

__global__ void k_trunc_flag(int64_t G2, const int32_t* __restrict__ slot, const double* __restrict__ leafnorm,
                             double tau2, int32_t* __restrict__ flag) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= G2) return;
  flag[m] = (slot[m] >= 0 && leafnorm[m] <= tau2) ? 1 : 0;
}

__global__ void k_trunc_compact(int64_t G2, const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                                const double* __restrict__ leafnorm, double* __restrict__ cs,
                                int32_t* __restrict__ cm) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= G2 || !flag[m]) return;
  cs[pos[m]] = leafnorm[m];
  cm[pos[m]] = int32_t(m);
}

constexpr int kSelThreads = 1024;
constexpr int kSelLds = 4096;  // candidates cached in LDS when they fit

__device__ __forceinline__ bool key_le(uint64_t sb, uint32_t m, uint64_t khi, uint32_t klo) {
  return sb < khi || (sb == khi && m <= klo);
}

__global__ void __launch_bounds__(kSelThreads) k_trunc_select(const int64_t* __restrict__ mc_ptr,
                                                              const double* __restrict__ cs,
                                                              const int32_t* __restrict__ cm, int key_bits_lo,
                                                              double tau2, uint64_t* __restrict__ kout,
                                                              double* __restrict__ result) {
  __shared__ double red[kSelThreads / kWave];
  __shared__ double s_lds[kSelLds];
  __shared__ uint32_t m_lds[kSelLds];
  const int64_t mc = *mc_ptr;
  const bool cached = mc <= kSelLds;
  if (cached) {
    for (int64_t i = threadIdx.x; i < mc; i += kSelThreads) {
      s_lds[i] = cs[i];
      m_lds[i] = uint32_t(cm[i]);
    }
  }
  __syncthreads();
  uint64_t khi = 0;
  uint32_t klo = 0;
  for (int b = 63 + key_bits_lo; b >= 0; --b) {
    uint64_t thi = khi;
    uint32_t tlo = klo;
    if (b >= key_bits_lo) thi |= (uint64_t(1) << (b - key_bits_lo));
    else tlo |= (uint32_t(1) << b);
    double part = 0.0;
    for (int64_t i = threadIdx.x; i < mc; i += kSelThreads) {
      const double s = cached ? s_lds[i] : cs[i];
      const uint32_t m = cached ? m_lds[i] : uint32_t(cm[i]);
      if (key_le(__double_as_longlong(s), m, thi, tlo)) part += s;
    }
    const double F = block_sum_f64(part, red);
    if (F <= tau2) {
      khi = thi;
      klo = tlo;
    }
    __syncthreads();
  }
  // final dropped sum and count for K*
  double part = 0.0;
  int64_t cnt = 0;
  for (int64_t i = threadIdx.x; i < mc; i += kSelThreads) {
    const double s = cached ? s_lds[i] : cs[i];
    const uint32_t m = cached ? m_lds[i] : uint32_t(cm[i]);
    if (key_le(__double_as_longlong(s), m, khi, klo)) {
      part += s;
      ++cnt;
    }
  }
  const double F = block_sum_f64(part, red);
  __shared__ int64_t cred[kSelThreads / kWave];
  cnt = wave_sum_i64(cnt);
  if (lane_id() == 0) cred[threadIdx.x / kWave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t c = 0;
    for (int w = 0; w < kSelThreads / kWave; ++w) c += cred[w];
    kout[0] = khi;
    kout[1] = klo;
    result[0] = F;
    result[1] = double(c);
  }
}

__global__ void k_trunc_apply(int64_t G2, const int32_t* __restrict__ slot, const double* __restrict__ leafnorm,
                              const int32_t* __restrict__ flag, const uint64_t* __restrict__ kst,
                              int32_t* __restrict__ out_slot, double* __restrict__ out_norm) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (m >= G2) return;
  const double s = leafnorm[m];
  const bool drop = flag[m] && key_le(__double_as_longlong(s), uint32_t(m), kst[0], uint32_t(kst[1]));
  out_slot[m] = drop ? -1 : slot[m];
  out_norm[m] = drop ? 0.0 : s;
}

size_t trunc_scratch_bytes(int G) {
  const int64_t G2 = int64_t(G) * G;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(G2 * 4) + al((G2 + 1) * 8) + al(G2 * 8) + al(G2 * 4) + al(16) + al(scan_scratch_bytes(G2));
}

hipError_t launch_trunc(hipStream_t s, int G, const int32_t* slot, const double* leafnorm, double tau2,
                        int32_t* out_slot, double* out_leafnorm, void* scratch, size_t scratch_bytes,
                        double* result_dev) {
  const int64_t G2 = int64_t(G) * G;
  if (scratch_bytes < trunc_scratch_bytes(G)) return hipErrorInvalidValue;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  char* p = static_cast<char*>(scratch);
  int32_t* flag = reinterpret_cast<int32_t*>(p);
  p += al(G2 * 4);
  int64_t* pos = reinterpret_cast<int64_t*>(p);
  p += al((G2 + 1) * 8);
  double* cs = reinterpret_cast<double*>(p);
  p += al(G2 * 8);
  int32_t* cm = reinterpret_cast<int32_t*>(p);
  p += al(G2 * 4);
  uint64_t* kst = reinterpret_cast<uint64_t*>(p);
  p += al(16);
  const uint32_t nb = uint32_t((G2 + 255) / 256);
  hipLaunchKernelGGL(k_trunc_flag, dim3(nb), dim3(256), 0, s, G2, slot, leafnorm, tau2, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int32_t* dummy = nullptr;
  (void)dummy;
  // exclusive positions of the candidates; pos[G2] = candidate count
  const int64_t nbs = std::max<int64_t>(1, (G2 + kScanTile - 1) / kScanTile);
  int64_t* sums = reinterpret_cast<int64_t*>(p);
  hipLaunchKernelGGL((k_scan_tiles<int32_t>), dim3(uint32_t(nbs)), dim3(kScanThreads), 0, s, flag, G2, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, sums, nbs, pos + G2);
  hipLaunchKernelGGL((k_scan_apply<int32_t, 0>), dim3(uint32_t(nbs)), dim3(kScanThreads), 0, s, flag, G2, sums,
                     pos, nullptr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trunc_compact, dim3(nb), dim3(256), 0, s, G2, flag, pos, leafnorm, cs, cm);
  int key_bits_lo = 1;
  while ((int64_t(1) << key_bits_lo) < G2) ++key_bits_lo;
  hipLaunchKernelGGL(k_trunc_select, dim3(1), dim3(kSelThreads), 0, s, pos + G2, cs, cm, key_bits_lo, tau2, kst,
                     result_dev);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trunc_apply, dim3(nb), dim3(256), 0, s, G2, slot, leafnorm, flag, kst, out_slot,
                     out_leafnorm);
  return hipGetLastError();
}

}  // namespace spamm
