// LDS-staged exclusive prefix scans, and input truncation with a global
// Frobenius budget (leaf-block form of Sec. 3's vector-space truncation).
#include "internal.h"
#include "kern_common.h"

namespace spamm {

constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;
constexpr int64_t kDirectTiles = 1024;  // up to this many tiles, two launches instead of three

// ---------------------------------------------------------------- scan

// Scan inputs are read through a source functor (element i -> int64 value)
// and every element's exclusive prefix may also go to a sink functor, so that
// a producer or a consumer pass can ride along with the scan's own launches.
template <typename In>
struct ArraySrc {
  const In* p;
  __device__ int64_t operator()(int64_t i) const { return int64_t(p[i]); }
};
struct NoSink {
  __device__ void operator()(int64_t, int64_t, int64_t) const {}
};

template <typename Src>
__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const Src src, int64_t count,
                                                            int64_t* __restrict__ sums) {
  __shared__ int64_t red[kScanThreads / kWave];
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  int64_t v = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + int64_t(i) * kScanThreads + threadIdx.x;
    if (idx < count) v += src(idx);
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
  if (threadIdx.x == 0 && total) *total = carry_sh;
}

// mode 0: out64[i] = exclusive prefix; mode 1: out32[i] = in[i] ? prefix : -1
// and, with keys, keys[prefix] = i for the flagged i (the inverse map).
// Direct (few tiles): each tile adds up the sums of the tiles before it
// itself (integer sums, exact in any order) and the last tile writes the
// total, so no separate pass over the tile sums is launched.
template <typename Src, int Mode, bool Direct, typename Sink>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const Src src, int64_t count,
                                                            const int64_t* __restrict__ offs,
                                                            int64_t* __restrict__ out64,
                                                            int32_t* __restrict__ out32,
                                                            int32_t* __restrict__ keys,
                                                            int64_t* __restrict__ total, const Sink sink) {
  __shared__ int64_t wtot[kScanThreads / kWave];
  __shared__ int64_t pre_sh[kScanThreads / kWave];
  int64_t tile_pre = 0;
  if constexpr (Direct) {
    int64_t acc = 0;
    for (int64_t j = threadIdx.x; j < int64_t(blockIdx.x); j += kScanThreads) acc += offs[j];
    acc = wave_sum_i64(acc);
    if (lane_id() == 0) pre_sh[threadIdx.x / kWave] = acc;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) tile_pre += pre_sh[w];
  } else {
    tile_pre = offs[blockIdx.x];
  }
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  int64_t vals[kScanItems];
  int64_t local = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    vals[i] = idx < count ? src(idx) : 0;
    local += vals[i];
  }
  const int64_t inc = wave_incl_scan(local);
  if (lane_id() == kWave - 1) wtot[threadIdx.x / kWave] = inc;
  __syncthreads();
  int64_t run = tile_pre + inc - local;
  for (int w = 0; w < int(threadIdx.x / kWave); ++w) run += wtot[w];
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < count) {
      if (Mode == 0) {
        if (out64) out64[idx] = run;
      } else {
        out32[idx] = vals[i] ? int32_t(run) : -1;
        if (keys && vals[i]) keys[run] = int32_t(idx);
      }
      sink(idx, vals[i], run);
    }
    run += vals[i];
  }
  if (Direct && total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) *total = run;
}

size_t scan_scratch_bytes(int64_t count) {
  const int64_t nb = (count + kScanTile - 1) / kScanTile;
  return size_t((nb + 1) * sizeof(int64_t) + 256);
}

template <int Mode, typename Src, typename Sink = NoSink>
static hipError_t scan_impl(hipStream_t s, const Src in, int64_t count, int64_t* out64, int32_t* out32,
                            int32_t* keys, int64_t* total, void* scratch, size_t scratch_bytes,
                            const Sink sink = Sink()) {
  const int64_t nb = std::max<int64_t>(1, (count + kScanTile - 1) / kScanTile);
  if (scratch_bytes < size_t(nb * sizeof(int64_t))) return hipErrorInvalidValue;
  int64_t* sums = static_cast<int64_t*>(scratch);
  hipLaunchKernelGGL((k_scan_tiles<Src>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, s, in, count, sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nb <= kDirectTiles) {
    hipLaunchKernelGGL((k_scan_apply<Src, Mode, true, Sink>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, s,
                       in, count, sums, out64, out32, keys, total, sink);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, sums, nb, total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_scan_apply<Src, Mode, false, Sink>), dim3(uint32_t(nb)), dim3(kScanThreads), 0, s, in,
                     count, sums, out64, out32, keys, total, sink);
  return hipGetLastError();
}

hipError_t launch_scan_i64(hipStream_t s, const int64_t* in, int64_t* out, int64_t count, void* scratch,
                           size_t scratch_bytes) {
  return scan_impl<0>(s, ArraySrc<int64_t>{in}, count, out, nullptr, nullptr, out + count, scratch, scratch_bytes);
}

hipError_t launch_flags_to_slots(hipStream_t s, const int32_t* flag, int64_t count, int32_t* slot, int32_t* keys,
                                 int64_t* total, void* scratch, size_t scratch_bytes) {
  return scan_impl<1>(s, ArraySrc<int32_t>{flag}, count, nullptr, slot, keys, total, scratch, scratch_bytes);
}

// ---------------------------------------------------------------- truncation
//
// Order the non-null leaves by the key (bits of the squared norm s, Morton
// index m) -- for s >= 0 the IEEE bit pattern orders like the value -- and
// drop the longest prefix whose summed squared norm is <= tau^2.  Only leaves
// with s <= tau^2 can be in that prefix (candidates).  For each candidate x,
// F(x) = sum of s_y over candidates y with key_y <= key_x, summed in one
// fixed order that does not depend on x (lane l of a wave adds the candidates
// y = l, l + 64, ... in index order, then a fixed tree adds the 64 lane sums).
// Rounding is monotone, so each addition only grows with x's key: F is
// monotone in the key and {x : F(x) <= tau^2} is a prefix of the order.
// Small candidate sets evaluate F(x) for every x from LDS; large ones build
// the largest admissible key bit by bit (F of each trial key summed in the
// workgroup's own fixed order, again monotone in the key).
// All jobs of a batch share one set of launches.

__device__ __forceinline__ int find_job(const TruncJob* __restrict__ jobs, int njobs, int64_t g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].base <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ bool key_le(uint64_t sb, uint32_t m, uint64_t khi, uint32_t klo) {
  return sb < khi || (sb == khi && m <= klo);
}

// The unit a leaf is truncated with: itself, or in the mirror-pair form its
// pair, represented by the leaf on or above the diagonal (rep), with weight
// s_rep + s_mirror (s of a null leaf is 0; a diagonal leaf is alone).
struct TruncUnit {
  uint32_t rep;
  double w;
  bool present;
};

__device__ __forceinline__ TruncUnit trunc_unit(const TruncJob& J, uint32_t m) {
  TruncUnit u;
  if (!J.pairs) {
    u.rep = m;
    u.present = J.slot[m] >= 0;
    u.w = J.leafnorm[m];
    return u;
  }
  uint32_t i, k;
  demorton(m, i, k);
  const uint32_t hi = i <= k ? m : morton(k, i), lo = morton(i <= k ? k : i, i <= k ? i : k);
  u.rep = hi;
  if (hi == lo) {
    u.present = J.slot[hi] >= 0;
    u.w = J.leafnorm[hi];
  } else {
    u.present = J.slot[hi] >= 0 || J.slot[lo] >= 0;
    u.w = J.leafnorm[hi] + J.leafnorm[lo];
  }
  return u;
}

// Non-null leaves of the unit represented by candidate m (the count that
// leaves the matrix when the unit is dropped).
__device__ __forceinline__ int64_t unit_leaves(const TruncJob& J, uint32_t m) {
  if (!J.pairs) return 1;  // (a candidate leaf is non-null)
  uint32_t i, k;
  demorton(m, i, k);
  return int64_t(J.slot[m] >= 0) + int64_t(i != k && J.slot[morton(k, i)] >= 0);
}

// Candidates (units with a non-null leaf and weight <= tau^2) are flagged,
// scanned, and compacted into (weight, Morton index) lists by the scan's
// sink, which looks up the job of flagged entries only.  In the pair form
// only the representative leaf of a pair is a candidate.
__global__ void k_trunc_flag(const TruncJob* __restrict__ jobs, int njobs, int64_t total, int32_t* __restrict__ flag) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const TruncJob& J = jobs[find_job(jobs, njobs, g)];
  const uint32_t m = uint32_t(g - J.base);
  const TruncUnit u = trunc_unit(J, m);
  flag[g] = (u.rep == m && u.present && u.w <= J.tau2) ? 1 : 0;
}

struct TruncCompactSink {
  const TruncJob* jobs;
  int njobs;
  double* cs;
  int32_t* cm;
  __device__ void operator()(int64_t g, int64_t v, int64_t pos) const {
    if (!v) return;
    const TruncJob& J = jobs[find_job(jobs, njobs, g)];
    const uint32_t m = uint32_t(g - J.base);
    cs[pos] = trunc_unit(J, m).w;
    cm[pos] = int32_t(m);
  }
};

constexpr int kSelThreads = 1024;
constexpr int kSelLds = 4096;   // candidate sets up to this size use the all-pairs form
constexpr int kSelSplit = 16;   // workgroups per job in the all-pairs form

// All-pairs form, part 1: the waves of a job's kSelSplit workgroups take the
// candidates x in turn; the lanes of a wave split the sum over y.
__global__ void __launch_bounds__(kSelThreads) k_trunc_fx(const TruncJob* __restrict__ jobs,
                                                          const int64_t* __restrict__ pos,
                                                          const double* __restrict__ cs_all,
                                                          const int32_t* __restrict__ cm_all,
                                                          double* __restrict__ fx_all) {
  __shared__ double s_lds[kSelLds];
  __shared__ uint32_t m_lds[kSelLds];
  const int job = blockIdx.x / kSelSplit, part = blockIdx.x % kSelSplit;
  const TruncJob& J = jobs[job];
  const int64_t c0 = pos[J.base];
  const int64_t mc = pos[J.base + int64_t(J.G) * J.G] - c0;
  if (mc > kSelLds || mc == 0) return;
  for (int64_t t = threadIdx.x; t < mc; t += kSelThreads) {
    s_lds[t] = cs_all[c0 + t];
    m_lds[t] = uint32_t(cm_all[c0 + t]);
  }
  __syncthreads();
  constexpr int NW = kSelThreads / kWave;
  const int w = threadIdx.x / kWave, lane = lane_id();
  for (int64_t x = int64_t(part) * NW + w; x < mc; x += int64_t(kSelSplit) * NW) {
    const uint64_t xh = __double_as_longlong(s_lds[x]);
    const uint32_t xl = m_lds[x];
    double f = 0.0;
#pragma unroll 4
    for (int64_t y = lane; y < mc; y += kWave) {
      const double sy = s_lds[y];
      if (key_le(__double_as_longlong(sy), m_lds[y], xh, xl)) f += sy;
    }
    f = wave_sum_f64(f);
    if (lane == 0) fx_all[c0 + x] = f;
  }
}

// Part 2 (and the large form): one workgroup per job picks the drop set.
__global__ void __launch_bounds__(kSelThreads) k_trunc_select(const TruncJob* __restrict__ jobs,
                                                              const int64_t* __restrict__ pos,
                                                              const double* __restrict__ cs_all,
                                                              const int32_t* __restrict__ cm_all,
                                                              const double* __restrict__ fx_all,
                                                              uint64_t* __restrict__ kst) {
  __shared__ double red[kSelThreads / kWave];
  __shared__ int64_t ired[kSelThreads / kWave];
  __shared__ uint64_t best_hi[kSelThreads / kWave];
  __shared__ uint32_t best_lo[kSelThreads / kWave];
  const TruncJob& J = jobs[blockIdx.x];
  const int64_t c0 = pos[J.base];
  const int64_t mc = pos[J.base + int64_t(J.G) * J.G] - c0;
  const double* cs = cs_all + c0;
  const int32_t* cm = cm_all + c0;
  const double tau2 = J.tau2;
  uint64_t khi = 0;
  uint32_t klo = 0;
  double F = 0.0;
  int64_t cnt = 0;
  if (mc <= kSelLds) {
    // max key (and its F) over the candidates with F(x) <= tau^2, and their count
    uint64_t my_hi = 0;
    uint32_t my_lo = 0;
    double my_F = 0.0;
    int64_t my_cnt = 0;
    bool any = false;
    for (int64_t x = threadIdx.x; x < mc; x += kSelThreads) {
      const double f = fx_all[c0 + x];
      if (f <= tau2) {
        const uint64_t xh = __double_as_longlong(cs[x]);
        const uint32_t xl = uint32_t(cm[x]);
        my_cnt += unit_leaves(J, xl);
        if (!any || !key_le(xh, xl, my_hi, my_lo)) {
          my_hi = xh;
          my_lo = xl;
          my_F = f;
        }
        any = true;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const uint64_t oh = __shfl_down(my_hi, off, kWave);
      const uint32_t ol = __shfl_down(my_lo, off, kWave);
      const double of = __shfl_down(my_F, off, kWave);
      const int oa = __shfl_down(int(any), off, kWave);
      my_cnt += __shfl_down(my_cnt, off, kWave);
      if (oa && (!any || !key_le(oh, ol, my_hi, my_lo))) {
        my_hi = oh;
        my_lo = ol;
        my_F = of;
        any = true;
      }
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == 0) {
      best_hi[w] = any ? my_hi : 0;
      best_lo[w] = any ? my_lo : 0;
      red[w] = any ? my_F : -1.0;
      ired[w] = my_cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      bool found = false;
      for (int q = 0; q < kSelThreads / kWave; ++q) {
        cnt += ired[q];
        if (red[q] >= 0.0 && (!found || !key_le(best_hi[q], best_lo[q], khi, klo))) {
          khi = best_hi[q];
          klo = best_lo[q];
          F = red[q];
          found = true;
        }
      }
    }
  } else {
    for (int b = 63 + J.key_bits_lo; b >= 0; --b) {
      uint64_t thi = khi;
      uint32_t tlo = klo;
      if (b >= J.key_bits_lo) thi |= (uint64_t(1) << (b - J.key_bits_lo));
      else tlo |= (uint32_t(1) << b);
      double part = 0.0;
      for (int64_t i = threadIdx.x; i < mc; i += kSelThreads) {
        const double sv = cs[i];
        if (key_le(__double_as_longlong(sv), uint32_t(cm[i]), thi, tlo)) part += sv;
      }
      const double Ft = block_sum_f64(part, red);
      if (Ft <= tau2) {
        khi = thi;
        klo = tlo;
      }
      __syncthreads();
    }
    double part = 0.0;
    int64_t c = 0;
    for (int64_t i = threadIdx.x; i < mc; i += kSelThreads) {
      const double sv = cs[i];
      if (key_le(__double_as_longlong(sv), uint32_t(cm[i]), khi, klo)) {
        part += sv;
        c += unit_leaves(J, uint32_t(cm[i]));
      }
    }
    F = block_sum_f64(part, red);
    c = wave_sum_i64(c);
    if (lane_id() == 0) ired[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int q = 0; q < kSelThreads / kWave; ++q) cnt += ired[q];
  }
  if (threadIdx.x == 0) {
    // (non-null leaves dropped; zero means nothing is dropped)
    kst[3 * blockIdx.x] = khi;
    kst[3 * blockIdx.x + 1] = klo;
    kst[3 * blockIdx.x + 2] = uint64_t(cnt);
    J.result[0] = cnt ? F : 0.0;
    J.result[1] = double(cnt);
  }
}

__global__ void k_trunc_apply(const TruncJob* __restrict__ jobs, int njobs, int64_t total,
                              const uint64_t* __restrict__ kst) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int j = find_job(jobs, njobs, g);
  const TruncJob& J = jobs[j];
  const int64_t m = g - J.base;
  const double s = J.leafnorm[m];
  // a leaf goes with its unit (itself, or its mirror pair)
  const TruncUnit u = trunc_unit(J, uint32_t(m));
  const bool cand = u.present && u.w <= J.tau2;
  const bool drop = cand && kst[3 * j + 2] != 0 &&
                    key_le(__double_as_longlong(u.w), u.rep, kst[3 * j], uint32_t(kst[3 * j + 1]));
  J.out_slot[m] = drop ? -1 : J.slot[m];
  J.out_norm[m] = drop ? 0.0 : s;
}

static size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

size_t trunc_batch_scratch_bytes(int njobs, int64_t total) {
  return al256(total * 4) + al256((total + 1) * 8) + al256(total * 8) + al256(total * 4) + al256(total * 8) +
         al256(size_t(njobs) * 24) + al256(scan_scratch_bytes(total));
}

hipError_t launch_trunc_batch(hipStream_t s, const TruncJob* jobs, int njobs, int64_t total, void* scratch,
                              size_t scratch_bytes) {
  if (njobs == 0) return hipSuccess;
  if (scratch_bytes < trunc_batch_scratch_bytes(njobs, total)) return hipErrorInvalidValue;
  char* p = static_cast<char*>(scratch);
  int32_t* flag = reinterpret_cast<int32_t*>(p);
  p += al256(total * 4);
  int64_t* pos = reinterpret_cast<int64_t*>(p);
  p += al256((total + 1) * 8);
  double* cs = reinterpret_cast<double*>(p);
  p += al256(total * 8);
  int32_t* cm = reinterpret_cast<int32_t*>(p);
  p += al256(total * 4);
  double* fx = reinterpret_cast<double*>(p);
  p += al256(total * 8);
  uint64_t* kst = reinterpret_cast<uint64_t*>(p);
  p += al256(size_t(njobs) * 24);
  const uint32_t nb = uint32_t((total + 255) / 256);
  hipLaunchKernelGGL(k_trunc_flag, dim3(nb), dim3(256), 0, s, jobs, njobs, total, flag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_impl<0>(s, ArraySrc<int32_t>{flag}, total, pos, nullptr, nullptr, pos + total, p,
                   scan_scratch_bytes(total), TruncCompactSink{jobs, njobs, cs, cm});
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trunc_fx, dim3(uint32_t(njobs) * kSelSplit), dim3(kSelThreads), 0, s, jobs, pos, cs, cm, fx);
  hipLaunchKernelGGL(k_trunc_select, dim3(uint32_t(njobs)), dim3(kSelThreads), 0, s, jobs, pos, cs, cm, fx, kst);
  hipLaunchKernelGGL(k_trunc_apply, dim3(nb), dim3(256), 0, s, jobs, njobs, total, kst);
  return hipGetLastError();
}

}  // namespace spamm
