// Build-time kernels: leaf norms and null flags (Sec. 2, Sec. 4.2, Sec. 4.4),
// compaction into the leaf store (Morton order for a dense input, list order
// for a block list), derived compute copies, the row/column views used by
// pruning, and the squared-norm pyramid.
#include "internal.h"
#include "kern_common.h"

namespace spamm {

// error bits reported by the block-list build
constexpr int kErrCoord = 1, kErrDup = 2, kErrPad = 4;

// ---------------------------------------------------------------- leaf scan

// Leaf passes: thread t takes the elements t, t + 256, t + 512, ... of a leaf
// (row-major), kLeafPass of them per pass with every load issued before the
// first use.  The per-thread order is the same for every kernel below, so the
// dense and the block-list builds give bitwise equal norms.
constexpr int kLeafPass = 8;

// One workgroup per leaf (Morton index = blockIdx): FP64 squared norm (each
// thread sums its fixed strided share of the leaf, then a fixed tree), the
// non-zero flag and the non-finite flag.  Reads the dense input once.
__global__ void __launch_bounds__(256) k_build_scan_dense(const double* __restrict__ dense,
                                                          int64_t n, int64_t ld, int bs,
                                                          double* __restrict__ leafnorm,
                                                          int32_t* __restrict__ flag,
                                                          int32_t* __restrict__ nonfinite) {
  __shared__ double red[4];
  const uint32_t m = blockIdx.x;
  uint32_t r, c;
  demorton(m, r, c);
  const int64_t r0 = int64_t(r) * bs, c0 = int64_t(c) * bs;
  double s = 0.0;
  int nz = 0, nf = 0;
  if (r0 < n && c0 < n) {
    const int rows = int(min<int64_t>(bs, n - r0)), cols = int(min<int64_t>(bs, n - c0));
    const int sh = __builtin_ctz(unsigned(bs)), e2 = bs * bs;
    for (int base = 0; base < e2; base += kLeafPass * 256) {
      double a[kLeafPass];
#pragma unroll
      for (int q = 0; q < kLeafPass; ++q) {  // all loads of the pass first
        const int e = base + q * 256 + int(threadIdx.x);
        const int rr = e >> sh, cc = e & (bs - 1);
        a[q] = (e < e2 && rr < rows && cc < cols) ? dense[(r0 + rr) * ld + c0 + cc] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kLeafPass; ++q) {
        const int e = base + q * 256 + int(threadIdx.x);
        const int rr = e >> sh, cc = e & (bs - 1);
        if (e < e2 && rr < rows && cc < cols) {
          s += a[q] * a[q];
          nz |= (a[q] != 0.0);
          nf |= !isfinite(a[q]);
        }
      }
    }
  }
  s = block_sum_f64(s, red);
  nz = __syncthreads_or(nz);
  nf = __syncthreads_or(nf);
  if (threadIdx.x == 0) {
    leafnorm[m] = nz ? s : 0.0;
    flag[m] = nz;
    if (nf) atomicOr(nonfinite, 1);
  }
}

hipError_t launch_build_scan_dense(hipStream_t s, const double* dense, int64_t n, int64_t ld,
                                   int bs, int G, double* leafnorm, int32_t* flag,
                                   int32_t* nonfinite) {
  hipLaunchKernelGGL(k_build_scan_dense, dim3(uint32_t(G) * uint32_t(G)), dim3(256), 0, s, dense,
                     n, ld, bs, leafnorm, flag, nonfinite);
  return hipGetLastError();
}

// FP32 -> BF16 bits, round to nearest even (inputs are finite).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// One workgroup writes every requested copy of one leaf slot `sl` from the
// leaf's FP64 values (get(e) for row-major element e).  The split-BF16 pair
// is hi = bf16(x32), lo = bf16(x32 - hi) with x32 the FP32 rounding of the
// value.  The transposed BF16 copy goes through a 64 x 64 LDS tile so its
// stores stay coalesced.
template <typename Get>
__device__ __forceinline__ void write_leaf(int64_t sl, int bs, Get get, double* f64, float* f32, uint16_t* b16,
                                           uint16_t* b16t) {
  __shared__ uint32_t tile[64 * 65];
  const int64_t e2 = int64_t(bs) * bs;
  const int64_t base = sl * e2;
  for (int b0 = 0; b0 < e2; b0 += kLeafPass * 256) {
    double av[kLeafPass];
#pragma unroll
    for (int q = 0; q < kLeafPass; ++q) {  // all loads of the pass first
      const int e = b0 + q * 256 + int(threadIdx.x);
      av[q] = e < e2 ? get(e) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kLeafPass; ++q) {
      const int e = b0 + q * 256 + int(threadIdx.x);
      if (e >= e2) continue;
      const double a = av[q];
      if (f64) f64[base + e] = a;
      const float x = float(a);
      if (f32) f32[base + e] = x;
      if (b16) {
        const uint16_t h = f32_to_bf16(x);
        b16[2 * base + e] = h;
        b16[2 * base + e2 + e] = f32_to_bf16(x - bf16_to_f32(h));
      }
    }
  }
  if (!b16t) return;
  // transposed copy, 64 x 64 sub-tiles (one for bs <= 64)
  const int ts = bs < 64 ? bs : 64;
  for (int tr = 0; tr < bs; tr += ts)
    for (int tc = 0; tc < bs; tc += ts) {
      __syncthreads();
      for (int e = threadIdx.x; e < ts * ts; e += blockDim.x) {
        const int r = e / ts, c = e % ts;
        const float x = float(get((tr + r) * bs + tc + c));
        const uint16_t h = f32_to_bf16(x);
        const uint16_t l = f32_to_bf16(x - bf16_to_f32(h));
        tile[r * 65 + c] = uint32_t(h) | (uint32_t(l) << 16);
      }
      __syncthreads();
      // element (c, r) of the transposed leaf = element (r, c) of the leaf
      for (int e = threadIdx.x; e < ts * ts; e += blockDim.x) {
        const int c = e / ts, r = e % ts;
        const uint32_t v = tile[r * 65 + c];
        const int64_t o = int64_t(tc + c) * bs + tr + r;
        b16t[2 * base + o] = uint16_t(v & 0xffffu);
        b16t[2 * base + e2 + o] = uint16_t(v >> 16);
      }
    }
}

// ---------------------------------------------------------------- batched block lists

// The lists of one build call, each kernel over all of them; a thread or
// workgroup finds its list by the list's first index (G*G entries or blocks
// of the batch).
template <int Field>
__device__ __forceinline__ int find_bjob(const BuildJob* __restrict__ jobs, int njobs, int64_t g) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t b = Field == 0 ? jobs[mid].g2_base : jobs[mid].blk_base;
    if (b <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_build_init_b(const BuildJob* __restrict__ jobs, int njobs, int64_t g2_total) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= g2_total) return;
  const BuildJob& J = jobs[find_bjob<0>(jobs, njobs, g)];
  const int64_t m = g - J.g2_base;
  if (m < 4) J.err[m] = 0;
  if (m == 0) *J.total = 0;
  J.src_of[m] = -1;
  J.slot[m] = -1;
  J.leafnorm[m] = 0.0;
}

__global__ void k_blocks_scatter_b(const BuildJob* __restrict__ jobs, int njobs, int64_t blocks_total) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= blocks_total) return;
  const BuildJob& J = jobs[find_bjob<1>(jobs, njobs, g)];
  const int64_t t = g - J.blk_base;
  const int64_t gmax = (J.n + J.bs - 1) / J.bs;
  const int32_t I = J.coords[2 * t], Jc = J.coords[2 * t + 1];
  if (I < 0 || Jc < 0 || I >= gmax || Jc >= gmax) {
    atomicOr(J.err, kErrCoord);
    return;
  }
  const uint32_t m = morton(uint32_t(I), uint32_t(Jc));
  const int32_t old = atomicCAS(&J.src_of[m], -1, int32_t(t));
  if (old != -1) atomicOr(J.err, kErrDup);
}

// One workgroup per block of the batch.  The block that won its Morton slot
// gets its squared norm (the leaf-pass order of k_build_scan_dense, so both
// builds give the same bits) and, when it is not all zero, becomes leaf slot
// t of its list: slot map, key, leaf copies (read again from L2) and one
// count.  A list's store therefore has a slot per listed block, in list
// order; slots of zero or rejected blocks stay unused.
__global__ void __launch_bounds__(256) k_blocks_scan_b(const BuildJob* __restrict__ jobs, int njobs) {
  __shared__ double red[4];
  const BuildJob& J = jobs[find_bjob<1>(jobs, njobs, blockIdx.x)];
  const int64_t t = int64_t(blockIdx.x) - J.blk_base;
  const int bs = J.bs;
  const int64_t n = J.n;
  const int64_t gmax = (n + bs - 1) / bs;
  const int32_t I = J.coords[2 * t], Jc = J.coords[2 * t + 1];
  if (I < 0 || Jc < 0 || I >= gmax || Jc >= gmax) return;
  const uint32_t m = morton(uint32_t(I), uint32_t(Jc));
  if (J.src_of[m] != int32_t(t)) return;
  double s = 0.0;
  int nz = 0, nf = 0, pad = 0;
  const int64_t rows = min<int64_t>(bs, n - int64_t(I) * bs);
  const int64_t cols = min<int64_t>(bs, n - int64_t(Jc) * bs);
  const double* blk = J.data + t * bs * bs;
  const int sh = __builtin_ctz(unsigned(bs)), e2 = bs * bs;
  for (int base = 0; base < e2; base += kLeafPass * 256) {
    double a[kLeafPass];
#pragma unroll
    for (int q = 0; q < kLeafPass; ++q) {
      const int e = base + q * 256 + int(threadIdx.x);
      a[q] = e < e2 ? blk[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kLeafPass; ++q) {
      const int e = base + q * 256 + int(threadIdx.x);
      const int rr = e >> sh, cc = e & (bs - 1);
      if (e >= e2) continue;
      if (rr < rows && cc < cols) {
        s += a[q] * a[q];
        nz |= (a[q] != 0.0);
        nf |= !isfinite(a[q]);
      } else {
        pad |= (a[q] != 0.0);
      }
    }
  }
  s = block_sum_f64(s, red);
  nz = __syncthreads_or(nz);
  nf = __syncthreads_or(nf);
  pad = __syncthreads_or(pad);
  if (threadIdx.x == 0) {
    J.leafnorm[m] = nz ? s : 0.0;
    if (nz) {
      J.slot[m] = int32_t(t);
      J.keys[t] = int32_t(m);
      atomicAdd(reinterpret_cast<unsigned long long*>(J.total), 1ull);
    }
    if (nf) atomicOr(J.err, 8);
    if (pad) atomicOr(J.err, kErrPad);
  }
  if (nz) write_leaf(t, bs, [&](int e) { return blk[e]; }, J.f64, J.f32, J.b16, J.b16t);
}

// ---------------------------------------------------------------- compaction


__global__ void __launch_bounds__(256) k_copy_dense_leaves(const double* __restrict__ dense, int64_t n,
                                                           int64_t ld, int bs,
                                                           const int32_t* __restrict__ keys,
                                                           double* f64, float* f32, uint16_t* b16,
                                                           uint16_t* b16t) {
  const int64_t sl = blockIdx.x;
  uint32_t r, c;
  demorton(uint32_t(keys[sl]), r, c);
  const int64_t r0 = int64_t(r) * bs, c0 = int64_t(c) * bs;
  const int64_t rows = min<int64_t>(bs, n - r0), cols = min<int64_t>(bs, n - c0);
  const int sh = __builtin_ctz(unsigned(bs));
  write_leaf(
      sl, bs,
      [&](int e) {
        const int rr = e >> sh, cc = e & (bs - 1);
        return (rr < rows && cc < cols) ? dense[(r0 + rr) * ld + c0 + cc] : 0.0;
      },
      f64, f32, b16, b16t);
}

hipError_t launch_copy_dense_leaves(hipStream_t s, const double* dense, int64_t n, int64_t ld,
                                    int bs, int64_t nleaf, const int32_t* keys, double* f64,
                                    float* f32, uint16_t* b16, uint16_t* b16t) {
  if (nleaf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_dense_leaves, dim3(uint32_t(nleaf)), dim3(256), 0, s, dense, n, ld, bs,
                     keys, f64, f32, b16, b16t);
  return hipGetLastError();
}

hipError_t launch_build_batch(hipStream_t s, const BuildJob* jobs, int njobs, int64_t g2_total,
                              int64_t blocks_total) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_init_b, dim3(uint32_t((g2_total + 255) / 256)), dim3(256), 0, s, jobs, njobs, g2_total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || blocks_total == 0) return e;
  hipLaunchKernelGGL(k_blocks_scatter_b, dim3(uint32_t((blocks_total + 255) / 256)), dim3(256), 0, s, jobs, njobs,
                     blocks_total);
  hipLaunchKernelGGL(k_blocks_scan_b, dim3(uint32_t(blocks_total)), dim3(256), 0, s, jobs, njobs);
  return hipGetLastError();
}

// Element-wise truncation (the truncated matrix of Thm. 1): every entry with
// |a| < tau becomes zero.  One workgroup per leaf, over the slot map: the
// kept entries' squared norm and the dropped entries' squared norm in FP64, a
// leaf with no non-zero entry left becomes null, and the others keep their
// slot in a new store of the same size, with every copy written again.
__global__ void __launch_bounds__(256) k_trunc_elem(const ElemTruncJob J) {
  __shared__ double red[4];
  const int64_t G2 = int64_t(J.G) * J.G;
  const int bs = J.bs, e2 = bs * bs;
  const double tau = J.tau;
  for (int64_t m = blockIdx.x; m < G2; m += gridDim.x) {
    const int32_t t = J.in_slot[m];  // uniform over the workgroup
    if (t < 0) {
      if (threadIdx.x == 0) {
        J.slot[m] = -1;
        J.leafnorm[m] = 0.0;
        J.dropped[m] = 0.0;
      }
      continue;
    }
    const double* src = J.in_f64 + int64_t(t) * e2;
    double s = 0.0, d = 0.0;
    int nz = 0;
    for (int base = 0; base < e2; base += kLeafPass * 256) {
      double a[kLeafPass];
#pragma unroll
      for (int q = 0; q < kLeafPass; ++q) {
        const int e = base + q * 256 + int(threadIdx.x);
        a[q] = e < e2 ? src[e] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < kLeafPass; ++q) {
        const double x = a[q];
        const double xx = x * x;
        if (fabs(x) < tau) {
          d += xx;
        } else {
          s += xx;
          nz |= (x != 0.0);
        }
      }
    }
    s = block_sum_f64(s, red);
    d = block_sum_f64(d, red);
    nz = __syncthreads_or(nz);
    if (threadIdx.x == 0) {
      J.leafnorm[m] = nz ? s : 0.0;
      J.slot[m] = nz ? t : -1;
      J.dropped[m] = d;
      if (nz) atomicAdd(reinterpret_cast<unsigned long long*>(J.count), 1ull);
    }
    if (nz)
      write_leaf(t, bs, [&](int e) { const double x = src[e]; return fabs(x) < tau ? 0.0 : x; }, J.f64, J.f32,
                 J.b16, J.b16t);
    __syncthreads();  // red and the LDS tile are reused by the next leaf
  }
}

hipError_t launch_trunc_elem(hipStream_t s, const ElemTruncJob& job) {
  const int64_t G2 = int64_t(job.G) * job.G;
  hipLaunchKernelGGL(k_trunc_elem, dim3(uint32_t(G2 < 65536 ? G2 : 65536)), dim3(256), 0, s, job);
  return hipGetLastError();
}

// Sum of n doubles in one fixed order: chunks of 4096 (one workgroup each),
// then the chunk sums in order.
__global__ void __launch_bounds__(256) k_sum_chunks(const double* __restrict__ v, int64_t n,
                                                    double* __restrict__ partial) {
  __shared__ double red[4];
  const int64_t c0 = int64_t(blockIdx.x) * 4096, c1 = min<int64_t>(n, c0 + 4096);
  double s = 0.0;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) s += v[i];
  s = block_sum_f64(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void k_sum_final(const double* __restrict__ partial, int64_t nchunks, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int64_t q = 0; q < nchunks; ++q) s += partial[q];
  *out = s;
}

hipError_t launch_sum_f64(hipStream_t s, const double* v, int64_t n, double* partial, double* out) {
  const int64_t nchunks = (n + 4095) / 4096;
  if (nchunks > 0) {
    hipLaunchKernelGGL(k_sum_chunks, dim3(uint32_t(nchunks)), dim3(256), 0, s, v, n, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, s, partial, nchunks, out);
  return hipGetLastError();
}

// Derive missing copies of every leaf from the best copy present (FP64 if
// any), one workgroup per leaf.
__global__ void __launch_bounds__(256) k_derive_store(int64_t nleaf, int bs, const double* __restrict__ f64,
                                                      const float* __restrict__ f32, double* o64, float* o32,
                                                      uint16_t* o16, uint16_t* o16t) {
  const int64_t e2 = int64_t(bs) * bs;
  for (int64_t sl = blockIdx.x; sl < nleaf; sl += gridDim.x) {
    const double* a64 = f64 ? f64 + sl * e2 : nullptr;
    const float* a32 = f32 ? f32 + sl * e2 : nullptr;
    write_leaf(sl, bs, [&](int e) { return a64 ? a64[e] : double(a32[e]); }, o64, o32, o16, o16t);
    __syncthreads();  // the LDS tile is reused by the next leaf
  }
}

hipError_t launch_derive_store(hipStream_t s, int64_t nleaf, int bs, const double* f64, const float* f32,
                               double* o64, float* o32, uint16_t* o16, uint16_t* o16t) {
  if (nleaf == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(nleaf, 65536);
  hipLaunchKernelGGL(k_derive_store, dim3(uint32_t(blocks)), dim3(256), 0, s, nleaf, bs, f64, f32, o64, o32,
                     o16, o16t);
  return hipGetLastError();
}

// ---------------------------------------------------------------- pruning views

// Row-major and column-major copies of sqrt(leaf norm) (-1 for null) and of
// the slot map, so that pruning walks an A row and a B column contiguously;
// then the non-null k range of every row and column (one wave each).  Both
// passes cover all matrices of a batch.
__device__ __forceinline__ int find_prep(const PrepJob* __restrict__ jobs, int njobs, int64_t g, bool waves) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((waves ? jobs[mid].wbase : jobs[mid].base) <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One launch: the first nb_prep workgroups write the row-major and
// column-major views (one entry per thread); the others find, one wave per
// row or column, the k range of its non-null leaves from the slot map.
__global__ void __launch_bounds__(256) k_prep(const PrepJob* __restrict__ jobs, int njobs, int64_t total,
                                              int64_t total_waves, int64_t nb_prep) {
  if (int64_t(blockIdx.x) < nb_prep) {
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const PrepJob& J = jobs[find_prep(jobs, njobs, g, false)];
    const int64_t m = g - J.base;
    const int G = J.G;
    uint32_t r, c;
    demorton(uint32_t(m), r, c);
    const int32_t sl = J.slot[m];
    const double v = sl >= 0 ? sqrt(J.leafnorm[m]) : -1.0;
    J.rm_sqrt[int64_t(r) * G + c] = v;
    J.rm_slot[int64_t(r) * G + c] = sl;
    J.cm_sqrt[int64_t(c) * G + r] = v;
    J.cm_slot[int64_t(c) * G + r] = sl;
    return;
  }
  const int64_t w = (int64_t(blockIdx.x) - nb_prep) * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (w >= total_waves) return;
  const PrepJob& J = jobs[find_prep(jobs, njobs, w, true)];
  const int G = J.G;
  const int64_t lw = w - J.wbase;
  const bool is_col = lw >= G;
  const uint32_t idx = uint32_t(is_col ? lw - G : lw);
  int lo = G, hi = -1;
  for (int k = lane_id(); k < G; k += kWave) {
    const uint32_t m = is_col ? morton(uint32_t(k), idx) : morton(idx, uint32_t(k));
    if (J.slot[m] >= 0) {
      lo = min(lo, k);
      hi = max(hi, k);
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    lo = min(lo, __shfl_down(lo, off, kWave));
    hi = max(hi, __shfl_down(hi, off, kWave));
  }
  if (lane_id() == 0) {
    J.ranges[(is_col ? 2 : 0) * G + idx] = lo;
    J.ranges[(is_col ? 3 : 1) * G + idx] = hi;
  }
}

hipError_t launch_prep_batch(hipStream_t s, const PrepJob* jobs, int njobs, int64_t total, int64_t total_waves) {
  if (njobs == 0) return hipSuccess;
  const int64_t nb_prep = (total + 255) / 256, nb_rng = (total_waves + 3) / 4;
  hipLaunchKernelGGL(k_prep, dim3(uint32_t(nb_prep + nb_rng)), dim3(256), 0, s, jobs, njobs, total, total_waves,
                     nb_prep);
  return hipGetLastError();
}

// ---------------------------------------------------------------- pyramid

constexpr int kPyrSub = 5;  // a subtree workgroup reduces 4^5 = 1024 leaves

// Reduce `vals` (4^h entries of level `lev`, Morton) in LDS up h levels,
// writing each level to norms.  Parent = ((c0 + c1) + c2) + c3.
__device__ void pyr_reduce_lds(double* lds, int h, double* norms, int lev, int64_t first) {
  int64_t cnt = int64_t(1) << (2 * h);
  for (int step = 0; step < h; ++step) {
    const int64_t pc = cnt / 4;
    for (int64_t p = threadIdx.x; p < pc; p += blockDim.x) {
      const double v = ((lds[4 * p] + lds[4 * p + 1]) + lds[4 * p + 2]) + lds[4 * p + 3];
      lds[cnt + p] = v;  // stage after current level
    }
    __syncthreads();
    for (int64_t p = threadIdx.x; p < pc; p += blockDim.x) {
      const double v = lds[cnt + p];
      lds[p] = v;
    }
    __syncthreads();
    first /= 4;
    --lev;
    for (int64_t p = threadIdx.x; p < pc; p += blockDim.x) norms[level_offset(lev) + first + p] = lds[p];
    cnt = pc;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_pyr_sub(const PyrJob* __restrict__ jobs, int njobs) {
  __shared__ double lds[1024 + 256];
  int j = 0;
  while (j + 1 < njobs && int64_t(blockIdx.x) >= jobs[j + 1].block_base) ++j;
  const PyrJob job = jobs[j];
  const int64_t w = int64_t(blockIdx.x) - job.block_base;
  const int h = job.sub_levels;
  const int64_t cnt = int64_t(1) << (2 * h);
  const int64_t first = w * cnt;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x)
    lds[i] = job.norms[level_offset(job.L) + first + i];
  __syncthreads();
  pyr_reduce_lds(lds, h, job.norms, job.L, first);
}

__global__ void __launch_bounds__(256) k_pyr_top(const PyrJob* __restrict__ jobs) {
  __shared__ double lds[4096 + 1024];
  const PyrJob job = jobs[blockIdx.x];
  const int top = job.L - job.sub_levels;  // levels left above the subtrees
  if (top <= 0) return;
  const int64_t cnt = int64_t(1) << (2 * top);
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x)
    lds[i] = job.norms[level_offset(top) + i];
  __syncthreads();
  pyr_reduce_lds(lds, top, job.norms, top, 0);
}

// Subtrees of sub_levels levels, one workgroup each, then the levels above
// them, one workgroup per job (a second launch: a cross-workgroup handoff
// inside one launch would need device-scope fences, which write back the
// XCD's L2 and cost more than the launch).
hipError_t launch_pyramid(hipStream_t s, const PyrJob* jobs_dev, int njobs, const std::vector<PyrJob>& jobs_host) {
  if (njobs == 0) return hipSuccess;
  int64_t blocks = 0;
  bool any_top = false;
  for (auto& jb : jobs_host) {
    blocks += jb.nsub;
    any_top |= jb.L > jb.sub_levels;
  }
  hipLaunchKernelGGL(k_pyr_sub, dim3(uint32_t(blocks)), dim3(256), 0, s, jobs_dev, njobs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !any_top) return e;
  hipLaunchKernelGGL(k_pyr_top, dim3(uint32_t(njobs)), dim3(256), 0, s, jobs_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dense out

__global__ void __launch_bounds__(256) k_to_dense(int64_t n, int bs, const int32_t* __restrict__ slot,
                                                  const double* __restrict__ f64,
                                                  const float* __restrict__ f32, double* out,
                                                  int64_t ld) {
  const uint32_t m = blockIdx.x;
  uint32_t r, c;
  demorton(m, r, c);
  const int64_t r0 = int64_t(r) * bs, c0 = int64_t(c) * bs;
  if (r0 >= n || c0 >= n) return;
  const int32_t sl = slot[m];
  const int64_t rows = min<int64_t>(bs, n - r0), cols = min<int64_t>(bs, n - c0);
  for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
    const int rr = e / bs, cc = e % bs;
    if (rr < rows && cc < cols) {
      double v = 0.0;
      if (sl >= 0) v = f64 ? f64[int64_t(sl) * bs * bs + e] : double(f32[int64_t(sl) * bs * bs + e]);
      out[(r0 + rr) * ld + c0 + cc] = v;
    }
  }
}

hipError_t launch_to_dense(hipStream_t s, int64_t n, int bs, int G, const int32_t* slot,
                           const double* f64, const float* f32, double* out, int64_t ld) {
  hipLaunchKernelGGL(k_to_dense, dim3(uint32_t(G) * uint32_t(G)), dim3(256), 0, s, n, bs, slot, f64,
                     f32, out, ld);
  return hipGetLastError();
}

// Leaves (ij[2t], ij[2t+1]) of a matrix into out[t * bs^2 ...] as FP64.
__global__ void __launch_bounds__(256) k_gather_leaves(int bs, const int32_t* __restrict__ slot,
                                                       const double* __restrict__ f64,
                                                       const float* __restrict__ f32,
                                                       const int32_t* __restrict__ ij, double* out) {
  const int64_t t = blockIdx.x;
  const int32_t sl = slot[morton(uint32_t(ij[2 * t]), uint32_t(ij[2 * t + 1]))];
  const int64_t e2 = int64_t(bs) * bs;
  for (int e = threadIdx.x; e < bs * bs; e += blockDim.x) {
    double v = 0.0;
    if (sl >= 0) v = f64 ? f64[sl * e2 + e] : double(f32[sl * e2 + e]);
    out[t * e2 + e] = v;
  }
}

hipError_t launch_gather_leaves(hipStream_t s, int bs, int64_t count, const int32_t* slot, const double* f64,
                                const float* f32, const int32_t* ij, double* out) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_leaves, dim3(uint32_t(count)), dim3(256), 0, s, bs, slot, f64, f32, ij, out);
  return hipGetLastError();
}

// Gershgorin discs, one workgroup per leaf row: every row i < n of the
// leaf row gets lo_i = a_ii - sum_{j != i} |a_ij| and hi_i = a_ii + sum; the
// workgroup keeps the min / max of its rows in part[2 * I], part[2 * I + 1]
// (rows past n are padding and are skipped).
__global__ void __launch_bounds__(256) k_gersh_rows(int64_t n, int bs, int G, const int32_t* __restrict__ slot,
                                                    const double* __restrict__ f64, const float* __restrict__ f32,
                                                    double* __restrict__ part) {
  __shared__ double rad[256], dia[256];
  __shared__ double mn[256], mx[256];
  const int I = blockIdx.x;
  const int tpr = blockDim.x / bs;  // threads per row (bs <= 256)
  const int r = threadIdx.x % bs, q = threadIdx.x / bs;
  const int64_t e2 = int64_t(bs) * bs;
  double s = 0.0, d = 0.0;
  for (int J = 0; J < G; ++J) {
    const int32_t sl = slot[morton(uint32_t(I), uint32_t(J))];
    if (sl < 0) continue;
    for (int c = q; c < bs; c += tpr) {
      const int64_t e = sl * e2 + int64_t(r) * bs + c;
      const double v = f64 ? f64[e] : double(f32[e]);
      if (J == I && c == r) d = v;
      else s += fabs(v);
    }
  }
  rad[threadIdx.x] = s;
  dia[threadIdx.x] = d;
  __syncthreads();
  double lo = 1e308, hi = -1e308;
  if (q == 0 && threadIdx.x < bs) {
    double rs = 0.0, dd = 0.0;
    for (int t = 0; t < tpr; ++t) {
      rs += rad[r + t * bs];
      dd += dia[r + t * bs];
    }
    if (int64_t(I) * bs + r < n) {
      lo = dd - rs;
      hi = dd + rs;
    }
  }
  mn[threadIdx.x] = lo;
  mx[threadIdx.x] = hi;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 1e308, b = -1e308;
    for (int t = 0; t < bs; ++t) {
      a = fmin(a, mn[t]);
      b = fmax(b, mx[t]);
    }
    part[2 * I] = a;
    part[2 * I + 1] = b;
  }
}

__global__ void k_gersh_final(int G, const double* __restrict__ part, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a = 1e308, b = -1e308;
  for (int I = 0; I < G; ++I) {
    a = fmin(a, part[2 * I]);
    b = fmax(b, part[2 * I + 1]);
  }
  out[0] = a;
  out[1] = b;
}

hipError_t launch_gershgorin(hipStream_t s, int64_t n, int bs, int G, const int32_t* slot, const double* f64,
                             const float* f32, double* part, double* out) {
  hipLaunchKernelGGL(k_gersh_rows, dim3(uint32_t(G)), dim3(256), 0, s, n, bs, G, slot, f64, f32, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(64), 0, s, G, part, out);
  return hipGetLastError();
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t value) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t count, int32_t value) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(uint32_t((count + 255) / 256)), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_zero_i32(hipStream_t s, int32_t* p, int64_t count) { return launch_fill_i32(s, p, count, 0); }

}  // namespace spamm
