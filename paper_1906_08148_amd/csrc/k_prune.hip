// Pruning: which leaf products are formed (Alg. 1's norm test with Alg. 2's
// null rule).  For every C leaf (i, j) the k range where A's row i and B's
// column j both have non-null leaves is walked, and k is kept when A_ik and
// B_kj are non-null and (SpAMM, Hybrid) sqrt(s_ik) * sqrt(s_kj) >= tau in
// FP64.  Because a parent's squared norm is a sum of non-negative terms,
// every ancestor of a kept triple passes the same test, so this flat test
// selects exactly the leaf products reached by the recursion of Alg. 1.
// The skipped products of each C leaf are summed k ascending (the bound
// b_ij of the error estimate).
//
// Counting pass -> LDS-staged exclusive scan over all C leaves of the batch
// (Morton order) -> fill pass writing the pairs (A and B leaf indices from
// the arena base), the C slot map and the GEMM work units.  No atomics:
// positions come from the scan, so the lists are deterministic.
#include "internal.h"
#include "kern_common.h"

namespace spamm {

__device__ __forceinline__ int64_t cnt_mask(int cb) { return (int64_t(1) << cb) - 1; }

// Requests' first global C index, cached in LDS by every workgroup (larger
// batches search the descriptor table in memory).
constexpr int kReqLds = 512;

__device__ __forceinline__ void cache_cbase(const ReqDev* __restrict__ reqs, int nreq, int64_t* sc) {
  for (int t = threadIdx.x; t < min(nreq, kReqLds); t += blockDim.x) sc[t] = reqs[t].cbase;
  __syncthreads();
}

__device__ __forceinline__ int find_req(const ReqDev* __restrict__ reqs, const int64_t* sc, int nreq, int64_t g) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((nreq <= kReqLds ? sc[mid] : reqs[mid].cbase) <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Each wave takes 64 consecutive C leaves (one per lane).  Every lane finds
// its request, intersects the k ranges of its A row and B column and keeps
// the base addresses of that row and column in the row-major / column-major
// prune views.  The wave then lays the k ranges of its 64 leaves end to end
// (a prefix sum of their lengths) and walks that flattened list with every
// lane busy: element t belongs to the leaf whose segment holds t (a binary
// search over the segment starts in LDS), and kPU elements per lane are
// loaded before any is used, so one round trip to memory serves up to
// kPU * 64 (leaf, k) candidates whatever the leaves' range lengths.  In the
// counting pass a wave whose longest range exceeds kLongSpan instead lets
// every lane walk its own leaf: the ranges are then long enough to keep the
// lanes busy, and a window of the flattened list would hold only one or two
// leaves, whose k-ordered sums would fall to one or two lanes.  Both walks
// add each leaf's terms k ascending, so they give the same bits.  The fill
// pass (no sums) always walks the flattened list, whose writes coalesce.
struct LaneLeaf {
  int r;
  uint32_t c, i, j;
  bool mirror;  // a symmetric square's leaf below the diagonal: walks its mirror (j, i)
  int lo, hi;
  const double* sa;  // sqrt norms of A's row i (index k)
  const double* sb;  // sqrt norms of B's column j
  const int32_t* la;  // slots of A's row i
  const int32_t* lb;  // slots of B's column j
  bool valid;
};

__device__ __forceinline__ LaneLeaf lane_leaf(const ReqDev* __restrict__ reqs, const int64_t* sc, int nreq,
                                              int64_t total_c, int64_t g) {
  LaneLeaf x;
  x.valid = g < total_c;
  x.r = 0;
  x.c = x.i = x.j = 0;
  x.mirror = false;
  x.lo = 1;
  x.hi = 0;
  x.sa = x.sb = nullptr;
  x.la = x.lb = nullptr;
  if (x.valid) {
    x.r = find_req(reqs, sc, nreq, g);
    const ReqDev& R = reqs[x.r];
    const int G = R.G;
    x.c = uint32_t(g - R.cbase);
    demorton(x.c, x.i, x.j);
    // a symmetric square decides a leaf below the diagonal as its mirror:
    // the same walk, so the same counts, bounds and kept set (transposed)
    x.mirror = R.sym && x.i > x.j && *R.asym == 0;
    const uint32_t wi = x.mirror ? x.j : x.i, wj = x.mirror ? x.i : x.j;
    x.lo = max(R.A.ranges[wi], R.B.ranges[2 * G + wj]);
    x.hi = min(R.A.ranges[G + wi], R.B.ranges[3 * G + wj]);
    x.sa = R.A.rm_sqrt + int64_t(wi) * G;
    x.sb = R.B.cm_sqrt + int64_t(wj) * G;
    x.la = R.A.rm_slot + int64_t(wi) * G;
    x.lb = R.B.cm_slot + int64_t(wj) * G;
  }
  return x;
}

constexpr int kLongSpan = 64;       // waves whose longest k range exceeds this walk one leaf per lane
constexpr int kPU = 8;              // flattened elements per lane per window
constexpr int kPW = kPU * kWave;    // window of the flattened list
constexpr int kPWaves = 4;          // waves per workgroup

__device__ __forceinline__ int wave_incl_scan_i32(int v) {
  const int l = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int o = __shfl_up(v, off, kWave);
    if (l >= off) v += o;
  }
  return v;
}
__device__ __forceinline__ int64_t wave_excl_scan_i64(int64_t v) {
  const int l = lane_id();
  int64_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int64_t o = __shfl_up(x, off, kWave);
    if (l >= off) x += o;
  }
  return x - v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, kWave));
  return v;
}

// LDS written by some lanes of a wave and read by others of the same wave:
// the workgroup-scope fences make the writes complete (lgkmcnt) and keep the
// compiler from moving accesses across; no other wave touches the region.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Owner of flattened element t < T: the last lane whose segment starts at or
// before t (lanes with empty segments share the next lane's start, so the
// last such lane has a non-empty segment holding t).
__device__ __forceinline__ int seg_owner(const int32_t* sst, int t) {
  int b = 0;
#pragma unroll
  for (int st = 32; st >= 1; st >>= 1)
    if (sst[b + st] <= t) b += st;
  return b;
}

struct CountLds {
  int32_t sst[kWave];
  int32_t lo[kWave];
  const double* sa[kWave];
  const double* sb[kWave];
  double tau[kWave];  // < 0: no norm test (Truncmul)
  double v[kPW];      // skipped product sqrt(s_ik) sqrt(s_kj), else 0
  uint8_t fl[kPW];    // bit 0: both leaves non-null, bit 1: kept
};

// Rounding coefficient of one C leaf summed from m kept products of order bs
// in precision prec: every entry of the computed sum lies within c * sum_k
// |A_ik| |B_kj| of the exact sum of those products.  c = e_in + gamma_n *
// mag: e_in bounds the representation error of the inputs in the compute
// precision (for a product of two inputs), gamma_n = n u / (1 - n u) the
// roundings of the sum along its longest chain (one product rounding, the
// bs - 1 additions of a leaf product, three times that for split BF16, and
// m additions across products), mag the size of the represented inputs.
__device__ double rounding_coef(int prec, int bs, int64_t m) {
  const double u64 = 0x1p-53, u32 = 0x1p-24, u16 = 0x1p-8;
  double e_in, mag, u, depth;
  if (prec == SPAMM_F64) {
    e_in = 0.0;
    mag = 1.0;
    u = u64;
    depth = double(bs + m + 1);
  } else if (prec == SPAMM_F32 || prec == SPAMM_BF16) {
    const double e = prec == SPAMM_F32 ? u32 : u32 + u16 * (1.0 + u32);  // FP64 -> FP32 (-> BF16)
    e_in = 2.0 * e + e * e;
    mag = (1.0 + e) * (1.0 + e);
    u = u32;
    depth = double(bs + m + 1);
  } else {
    const double e3 = u32 + u16 * u16 * (1.0 + u32);    // |hi + lo - x| <= e3 |x|
    const double el = (1.0 + u16) * u16 * (1.0 + u32);  // |lo| <= el |x|
    const double h = (1.0 + u16) * (1.0 + u32) + el;    // |hi| + |lo| <= h |x|
    e_in = 2.0 * e3 + e3 * e3 + el * el;                // lo_a lo_b is not formed
    mag = h * h;
    u = u32;
    depth = double(3 * bs + m + 1);
  }
  const double nu = depth * u;
  return e_in + nu / (1.0 - nu) * mag;
}

__global__ void __launch_bounds__(kPWaves * kWave) k_prune_count(const ReqDev* __restrict__ reqs, int nreq,
                                                                 int64_t total_c, int cb,
                                                                 int64_t* __restrict__ packed,
                                                                 double* __restrict__ bnd_all,
                                                                 int32_t* __restrict__ cand_all,
                                                                 double* __restrict__ pb_all) {
  __shared__ int64_t sc[kReqLds];
  __shared__ CountLds wl[kPWaves];
  cache_cbase(reqs, nreq, sc);
  const int64_t g0 = (int64_t(blockIdx.x) * kPWaves + threadIdx.x / kWave) * kWave;
  if (g0 >= total_c) return;
  const int lane = lane_id();
  const int64_t g = g0 + lane;
  const LaneLeaf x = lane_leaf(reqs, sc, nreq, total_c, g);
  CountLds& L = wl[threadIdx.x / kWave];
  const int span = (x.valid && x.lo <= x.hi) ? x.hi - x.lo + 1 : 0;
  const int incl = wave_incl_scan_i32(span);
  const int sst = incl - span;
  const int T = __builtin_amdgcn_readlane(incl, kWave - 1);
  int64_t my_cnt = 0, my_cand = 0;
  double my_skip = 0.0, my_kept = 0.0;  // skipped and kept norm products
  const int maxspan = wave_max_i32(span);
  if (maxspan > kLongSpan) {
    // long ranges: every lane walks its own leaf, k ascending, with eight
    // k values' loads in flight (the same order and arithmetic as below)
    const double tau = (x.valid && reqs[x.r].use_norms) ? reqs[x.r].tau : -1.0;
    for (int k0 = 0; k0 < maxspan; k0 += 8) {
      double a[8], bv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a[q] = bv[q] = -1.0;
        if (k0 + q < span) {
          a[q] = as_global(x.sa)[x.lo + k0 + q];
          bv[q] = as_global(x.sb)[x.lo + k0 + q];
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (k0 + q < span) {
          const bool both = (a[q] >= 0.0) && (bv[q] >= 0.0);
          const double pr = a[q] * bv[q];
          const bool keep = both && (tau < 0.0 || pr >= tau);
          my_cand += both ? 1 : 0;
          my_cnt += keep ? 1 : 0;
          my_skip += (both && !keep) ? pr : 0.0;
          my_kept += keep ? pr : 0.0;
        }
      }
    }
  } else if (T > 0) {
    L.sst[lane] = sst;
    L.lo[lane] = x.lo;
    L.sa[lane] = x.sa;
    L.sb[lane] = x.sb;
    L.tau[lane] = (x.valid && reqs[x.r].use_norms) ? reqs[x.r].tau : -1.0;
    wave_lds_sync();
    for (int wb = 0; wb < T; wb += kPW) {
      double a[kPU], bv[kPU];
      int own[kPU];
#pragma unroll
      for (int u = 0; u < kPU; ++u) {  // all loads of the window first
        const int t = wb + u * kWave + lane;
        a[u] = bv[u] = -1.0;
        own[u] = 0;
        if (t < T) {
          const int b = seg_owner(L.sst, t);
          const int k = L.lo[b] + (t - L.sst[b]);
          own[u] = b;
          a[u] = as_global(L.sa[b])[k];
          bv[u] = as_global(L.sb[b])[k];
        }
      }
#pragma unroll
      for (int u = 0; u < kPU; ++u) {
        const int t = wb + u * kWave + lane;
        if (t < T) {
          const double tau = L.tau[own[u]];
          const bool both = (a[u] >= 0.0) && (bv[u] >= 0.0);
          const double pr = a[u] * bv[u];
          const bool keep = both && (tau < 0.0 || pr >= tau);
          L.v[t - wb] = both ? pr : 0.0;
          L.fl[t - wb] = uint8_t((both ? 1 : 0) | (keep ? 2 : 0));
        }
      }
      wave_lds_sync();
      // each leaf adds its own part of the window, k ascending; eight LDS
      // reads are issued before their additions (long ranges leave a
      // window to one or two lanes)
      const int s0 = max(sst, wb) - wb, s1 = min(sst + span, wb + kPW) - wb;
      int t = s0;
      for (; t + 8 <= s1; t += 8) {
        double v[8];
        int f[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          v[q] = L.v[t + q];
          f[q] = L.fl[t + q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          my_cand += f[q] & 1;
          my_cnt += f[q] >> 1;
          my_skip += (f[q] & 2) ? 0.0 : v[q];
          my_kept += (f[q] & 2) ? v[q] : 0.0;
        }
      }
      for (; t < s1; ++t) {
        const int f = L.fl[t];
        const double v = L.v[t];
        my_cand += f & 1;
        my_cnt += f >> 1;
        my_skip += (f & 2) ? 0.0 : v;
        my_kept += (f & 2) ? v : 0.0;
      }
      wave_lds_sync();
    }
  }
  if (x.valid) {
    const ReqDev& R = reqs[x.r];
    const bool dflag = R.slotD != nullptr && R.slotD[x.c] >= 0;
    const int64_t flag = (my_cnt > 0 || dflag) ? 1 : 0;
    // a symmetric square forms no product below the diagonal: those leaves
    // are written from their mirrors (they keep their slot, bounds and counts)
    const int64_t formed = x.mirror ? 0 : my_cnt;
    packed[g] = (flag << cb) | formed;
    bnd_all[g] = my_skip;
    cand_all[g] = int32_t(my_cand);
    pb_all[g] = rounding_coef(R.prec, R.bs, my_cnt) * my_kept;
  }
}

hipError_t launch_prune_count(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c, int cnt_bits,
                              int64_t* packed, double* bnd_all, int32_t* cand_all, double* pb_all) {
  const int64_t waves = (total_c + kWave - 1) / kWave;
  const int64_t blocks = (waves + kPWaves - 1) / kPWaves;
  hipLaunchKernelGGL(k_prune_count, dim3(uint32_t(blocks)), dim3(kPWaves * kWave), 0, s, reqs, nreq, total_c,
                     cnt_bits, packed, bnd_all, cand_all, pb_all);
  return hipGetLastError();
}

__global__ void k_gather_totals(const ReqDev* __restrict__ reqs, int nreq, int cb,
                                const int64_t* __restrict__ scanned, ReqTotals* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nreq) return;
  const ReqDev& R = reqs[r];
  const int64_t a = scanned[R.cbase], b = scanned[R.cbase + int64_t(R.G) * R.G];
  out[r].n_kept = (b & cnt_mask(cb)) - (a & cnt_mask(cb));
  out[r].c_nonnull = (b >> cb) - (a >> cb);
}

hipError_t launch_gather_totals(hipStream_t s, const ReqDev* reqs, int nreq, int cnt_bits, const int64_t* scanned,
                                ReqTotals* out) {
  hipLaunchKernelGGL(k_gather_totals, dim3(uint32_t((nreq + 63) / 64)), dim3(64), 0, s, reqs, nreq, cnt_bits, scanned,
                     out);
  return hipGetLastError();
}

struct FillLds {
  int32_t sst[kWave];
  int32_t lo[kWave];
  const double* sa[kWave];
  const double* sb[kWave];
  const int32_t* la[kWave];
  const int32_t* lb[kWave];
  int64_t delta[kWave];
  int64_t beg[kWave];
  int64_t end[kWave];
  double tau[kWave];
  int2* out[kWave];
  int32_t* pk[kWave];  // k of each pair, or nullptr
  int32_t aoff[kWave];
  int32_t boff[kWave];
};

__global__ void __launch_bounds__(kPWaves * kWave) k_prune_fill(const ReqDev* __restrict__ reqs, int nreq,
                                                                int64_t total_c, int cb,
                                                                const int64_t* __restrict__ scanned,
                                                                const double* __restrict__ bnd_all,
                                                                const int32_t* __restrict__ cand_all,
                                                                WorkUnit* __restrict__ wu,
                                                                int64_t* __restrict__ cost) {
  __shared__ int64_t sc[kReqLds];
  __shared__ FillLds wl[kPWaves];
  cache_cbase(reqs, nreq, sc);
  const int64_t g0 = (int64_t(blockIdx.x) * kPWaves + threadIdx.x / kWave) * kWave;
  if (g0 >= total_c) return;
  const int lane = lane_id();
  const int64_t g = g0 + lane;
  const LaneLeaf x = lane_leaf(reqs, sc, nreq, total_c, g);
  int64_t off = 0, cnt = 0;
  if (x.valid) {
    const ReqDev& R = reqs[x.r];
    const int64_t G2 = int64_t(R.G) * R.G;
    const int64_t s0 = scanned[R.cbase], sg = scanned[g], s1 = scanned[g + 1];
    const int64_t cmk = cnt_mask(cb);
    off = (sg & cmk) - (s0 & cmk);
    cnt = (s1 & cmk) - (sg & cmk);
    const bool flag = ((s1 >> cb) - (sg >> cb)) != 0;
    const int32_t cs = int32_t((sg >> cb) - (s0 >> cb));
    R.off[x.c] = off;
    if (x.c == G2 - 1) R.off[G2] = off + cnt;
    R.cslot[x.c] = flag ? cs : -1;
    R.bnd[x.c] = bnd_all[g];
    R.ncand[x.c] = cand_all[g];
    if (flag) {
      R.ckeys[cs] = int32_t(x.c);
      // placement: slice q of every request's C leaves (Morton order) goes to
      // region q, which the workgroups of XCD q work through
      const int64_t cn = ((scanned[R.cbase + G2] >> cb) - (s0 >> cb));
      const int n = R.sched_n, ns = R.nslices;
      int q = 0;
      while (q + 1 < ns && cn * (q + 1) / ns <= cs) ++q;
      const int64_t* Q = R.sched + kXcds * (n + 1);  // offsets of the slices
      const int64_t at = Q[q] + R.sched[q * (n + 1) + R.sched_k] + (cs - cn * q / ns);
      if (at >= 0 && at < Q[kXcds]) {
        // a 256 leaf is four 128 x 128 tiles, one unit each, side by side
        const int nt = R.bs == 256 ? 4 : 1;
        WorkUnit u;
        u.pp = R.pairs_idx + off;
        u.cnt = int32_t(cnt);
        u.cidx = int32_t(R.cidx + cs);
        u.req = x.r;
        for (int t = 0; t < nt; ++t) {
          u.cflags = int32_t(x.c) | (R.use_ep ? kUnitEp : 0) | (t << kUnitTileShift);
          wu[R.wu_base + at * nt + t] = u;
          cost[R.wu_base + at * nt + t] = cnt + 1;
        }
      }
    } else {
      R.cnorm[level_offset(R.L) + x.c] = 0.0;
    }
    if (x.i == x.j) R.trace_part[x.i] = 0.0;
  }
  // the kept pairs of the wave's leaves, in flattened order; a running count
  // of kept elements gives each its place: leaf b's pairs start at off_b,
  // which is where the running count stands at b's segment start plus
  // delta_b = off_b - (kept elements of the earlier leaves of this wave)
  const int span = (x.valid && cnt > 0) ? x.hi - x.lo + 1 : 0;
  const int incl = wave_incl_scan_i32(span);
  const int sst = incl - span;
  const int T = __builtin_amdgcn_readlane(incl, kWave - 1);
  if (T == 0) return;
  FillLds& L = wl[threadIdx.x / kWave];
  const int64_t before = wave_excl_scan_i64(span > 0 ? cnt : 0);
  L.sst[lane] = sst;
  L.lo[lane] = x.lo;
  L.sa[lane] = x.sa;
  L.sb[lane] = x.sb;
  L.la[lane] = x.la;
  L.lb[lane] = x.lb;
  L.delta[lane] = off - before;
  L.beg[lane] = off;
  L.end[lane] = off + cnt;
  if (span > 0) {
    const ReqDev& R = reqs[x.r];
    L.tau[lane] = R.use_norms ? R.tau : -1.0;
    L.out[lane] = R.pairs;
    L.pk[lane] = R.pk;
    L.aoff[lane] = int32_t(R.aoff);
    L.boff[lane] = int32_t(R.boff);
  }
  wave_lds_sync();
  int64_t run = 0;  // kept elements before the current row of 64
  for (int wb = 0; wb < T; wb += kPW) {
    double a[kPU], bv[kPU];
    int32_t sa[kPU], sb[kPU], kk[kPU];
    int own[kPU];
#pragma unroll
    for (int u = 0; u < kPU; ++u) {  // norms and slots of the window in flight together
      const int t = wb + u * kWave + lane;
      a[u] = bv[u] = -1.0;
      sa[u] = sb[u] = 0;
      own[u] = 0;
      kk[u] = 0;
      if (t < T) {
        const int b = seg_owner(L.sst, t);
        const int k = L.lo[b] + (t - L.sst[b]);
        own[u] = b;
        kk[u] = k;
        a[u] = as_global(L.sa[b])[k];
        bv[u] = as_global(L.sb[b])[k];
        sa[u] = as_global(L.la[b])[k];
        sb[u] = as_global(L.lb[b])[k];
      }
    }
#pragma unroll
    for (int u = 0; u < kPU; ++u) {
      const int t = wb + u * kWave + lane;
      bool keep = false;
      int b = own[u];
      if (t < T) {
        const double tau = L.tau[b];
        const bool both = (a[u] >= 0.0) && (bv[u] >= 0.0);
        keep = both && (tau < 0.0 || a[u] * bv[u] >= tau);
      }
      const uint64_t mask = ballot64(keep);
      if (keep) {
        const int64_t at = L.delta[b] + run + popc64(mask & lanemask_lt());
        if (at >= L.beg[b] && at < L.end[b]) {
          L.out[b][at] = make_int2(L.aoff[b] + sa[u], L.boff[b] + sb[u]);
          if (L.pk[b]) L.pk[b][at] = kk[u];
        }
      }
      run += popc64(mask);
    }
  }
}

hipError_t launch_prune_fill(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c, int cnt_bits,
                             const int64_t* scanned, const double* bnd_all, const int32_t* cand_all,
                             WorkUnit* wu, int64_t* cost) {
  const int64_t waves = (total_c + kWave - 1) / kWave;
  const int64_t blocks = (waves + kPWaves - 1) / kPWaves;
  hipLaunchKernelGGL(k_prune_fill, dim3(uint32_t(blocks)), dim3(kPWaves * kWave), 0, s, reqs, nreq, total_c,
                     cnt_bits, scanned, bnd_all, cand_all, wu, cost);
  return hipGetLastError();
}

// Per-request accounting, reduced in one fixed order: partial sums over
// chunks of kStatChunk C leaves (one workgroup each), then one workgroup per
// request adds its partials in chunk order with the trace parts and gathers
// the pyramid roots and truncation results, so that one copy brings every
// statistic to the host.  The partial sums read the batch-wide skipped bounds
// and candidate counts of the counting pass (C leaf c of a request at cbase +
// c), so they can run before the fill pass.
__global__ void __launch_bounds__(256) k_stats_partial(const ReqDev* __restrict__ reqs, int nreq,
                                                       const double* __restrict__ bnd_all,
                                                       const int32_t* __restrict__ cand_all,
                                                       const double* __restrict__ pb_all,
                                                       StatPartial* __restrict__ partial) {
  __shared__ double red[4];
  __shared__ int64_t ired[4];
  int lo = 0, hi = nreq - 1;
  const int64_t chunk = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (reqs[mid].stat_base <= chunk) lo = mid;
    else hi = mid - 1;
  }
  const ReqDev& R = reqs[lo];
  const int64_t G2 = int64_t(R.G) * R.G;
  const int64_t c0 = (chunk - R.stat_base) * kStatChunk;
  const int64_t c1 = min<int64_t>(G2, c0 + kStatChunk);
  double b1 = 0.0, b2 = 0.0, b3 = 0.0;
  int64_t cand = 0;
  const double* bnd = bnd_all + R.cbase;
  const int32_t* ncand = cand_all + R.cbase;
  const double* pb = pb_all + R.cbase;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
    const double b = bnd[c];
    b1 += b;
    const double bb = b * b;
    b2 += bb;
    const double e = pb[c];
    const double ee = e * e;
    b3 += ee;
    cand += ncand[c];
  }
  b1 = block_sum_f64(b1, red);
  b2 = block_sum_f64(b2, red);
  b3 = block_sum_f64(b3, red);
  cand = wave_sum_i64(cand);
  __syncthreads();
  if (lane_id() == 0) ired[threadIdx.x / kWave] = cand;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < 4; ++w) t += ired[w];
    partial[chunk].b1 = b1;
    partial[chunk].b2 = b2;
    partial[chunk].pb = b3;
    partial[chunk].cand = t;
  }
}

__global__ void __launch_bounds__(256) k_stats_final(const ReqDev* __restrict__ reqs,
                                                     const StatPartial* __restrict__ partial,
                                                     ReqStatsDev* __restrict__ out) {
  __shared__ double red[4];
  const ReqDev& R = reqs[blockIdx.x];
  const int64_t G2 = int64_t(R.G) * R.G;
  const int64_t nch = (G2 + kStatChunk - 1) / kStatChunk;
  double tr = 0.0;
  for (int64_t i = threadIdx.x; i < R.G; i += blockDim.x) tr += R.trace_part[i];
  tr = block_sum_f64(tr, red);
  if (threadIdx.x == 0) {
    double b1 = 0.0, b2 = 0.0, b3 = 0.0;
    int64_t cand = 0;
    for (int64_t q = 0; q < nch; ++q) {
      b1 += partial[R.stat_base + q].b1;
      b2 += partial[R.stat_base + q].b2;
      b3 += partial[R.stat_base + q].pb;
      cand += partial[R.stat_base + q].cand;
    }
    ReqStatsDev o;
    o.B1 = b1;
    o.B2sq = b2;
    o.trace = tr;
    o.normC_sq = R.cnorm[0];
    o.normA_sq = *R.rootA;
    o.normB_sq = *R.rootB;
    o.normAu_sq = *R.rootAu;
    o.dA_sq = R.truncA ? R.truncA[0] : 0.0;
    o.dB_sq = R.truncB ? R.truncB[0] : 0.0;
    o.pb_sq = b3;
    o.n_candidates = cand;
    out[blockIdx.x] = o;
  }
}

hipError_t launch_stats_partial(hipStream_t s, const ReqDev* reqs, int nreq, int64_t nchunks,
                                const double* bnd_all, const int32_t* cand_all, const double* pb_all,
                                StatPartial* partial) {
  if (nreq == 0 || nchunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats_partial, dim3(uint32_t(nchunks)), dim3(256), 0, s, reqs, nreq, bnd_all, cand_all,
                     pb_all, partial);
  return hipGetLastError();
}

hipError_t launch_stats_final(hipStream_t s, const ReqDev* reqs, int nreq, const StatPartial* partial,
                              ReqStatsDev* out) {
  if (nreq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats_final, dim3(uint32_t(nreq)), dim3(256), 0, s, reqs, partial, out);
  return hipGetLastError();
}

// Symmetric squares (A = A^T, C = A A): the kept set is symmetric, because
// the norm product of (I, K, J) equals that of (J, K, I), and C_IJ = C_JI^T.
// Each non-null leaf below the diagonal is written as the transpose of its
// mirror through a 64 x 64 LDS tile, and takes the mirror's squared norm
// before the pyramid is summed.
template <typename T>
__device__ __forceinline__ void mirror_leaf(const T* __restrict__ src, T* __restrict__ dst, int bs, T* tile) {
  const int ts = bs < 64 ? bs : 64;
  for (int tr = 0; tr < bs; tr += ts)
    for (int tc = 0; tc < bs; tc += ts) {
      __syncthreads();
      // tile(r, c) = src(tc + r, tr + c); dst(tr + r, tc + c) = tile(c, r)
      for (int e = threadIdx.x; e < ts * ts; e += blockDim.x) {
        const int r = e / ts, c = e % ts;
        tile[r * (ts + 1) + c] = src[(tc + r) * bs + tr + c];
      }
      __syncthreads();
      for (int e = threadIdx.x; e < ts * ts; e += blockDim.x) {
        const int r = e / ts, c = e % ts;
        dst[(tr + r) * bs + tc + c] = tile[c * (ts + 1) + r];
      }
    }
}

__global__ void __launch_bounds__(256) k_mirror(const ReqDev* __restrict__ reqs, int nreq, int64_t total_c) {
  __shared__ double tile[64 * 65];
  for (int64_t g = blockIdx.x; g < total_c; g += gridDim.x) {  // uniform over the workgroup
    int lo = 0, hi = nreq - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (reqs[mid].cbase <= g) lo = mid;
      else hi = mid - 1;
    }
    const ReqDev& R = reqs[lo];
    if (!R.sym || *R.asym != 0) continue;  // not a symmetric square, or formed in full
    const uint32_t m = uint32_t(g - R.cbase);
    uint32_t I, J;
    demorton(m, I, J);
    if (I <= J) continue;
    const uint32_t m2 = morton(J, I);
    const int32_t sd = R.cslot[m], ss = R.cslot[m2];
    if (sd < 0 || ss < 0) continue;  // both null: the lower leaf took its mirror's decision
    const int64_t e2 = int64_t(R.bs) * R.bs;
    const int64_t lv = level_offset(R.L);
    if (threadIdx.x == 0) R.cnorm[lv + m] = R.cnorm[lv + m2];
    if (R.prec == SPAMM_F64) {
      const double* c = static_cast<const double*>(R.cstore);
      mirror_leaf(c + ss * e2, static_cast<double*>(R.cstore) + sd * e2, R.bs, tile);
    } else {
      const float* c = static_cast<const float*>(R.cstore);
      mirror_leaf(c + ss * e2, static_cast<float*>(R.cstore) + sd * e2, R.bs, reinterpret_cast<float*>(tile));
    }
  }
}

// Symmetry of a null map (and of the epilogue matrix's): one thread per
// leaf (I, K) with I < K compares it with (K, I); a wave with a mismatch
// sets the flag.
__global__ void k_sym_check(int G, const int32_t* __restrict__ slot, const int32_t* __restrict__ slotD,
                            int32_t* __restrict__ flag) {
  const int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  bool bad = false;
  if (m < int64_t(G) * G) {
    uint32_t I, K;
    demorton(uint32_t(m), I, K);
    if (I < K) {
      const uint32_t t = morton(K, I);
      bad = (slot[m] >= 0) != (slot[t] >= 0);
      if (slotD) bad = bad || ((slotD[m] >= 0) != (slotD[t] >= 0));
    }
  }
  if (__any(bad) && lane_id() == 0) atomicOr(flag, 1);
}

hipError_t launch_sym_check(hipStream_t s, int G, const int32_t* slot, const int32_t* slotD, int32_t* flag) {
  const int64_t G2 = int64_t(G) * G;
  hipLaunchKernelGGL(k_sym_check, dim3(uint32_t((G2 + 255) / 256)), dim3(256), 0, s, G, slot, slotD, flag);
  return hipGetLastError();
}

hipError_t launch_mirror(hipStream_t s, const ReqDev* reqs, int nreq, int64_t total_c) {
  if (nreq == 0 || total_c == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mirror, dim3(uint32_t(total_c < 16384 ? total_c : 16384)), dim3(256), 0, s, reqs, nreq,
                     total_c);
  return hipGetLastError();
}

// Squared Frobenius difference of a product's C and its FP64 twin's, in one
// fixed order: partial sums over chunks of kValChunk elements (one
// workgroup each), then each job adds its chunks in order.
__global__ void __launch_bounds__(256) k_val_partial(const ValJob* __restrict__ jobs, int njobs,
                                                     double* __restrict__ partial) {
  __shared__ double red[4];
  int lo = 0, hi = njobs - 1;
  const int64_t chunk = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].chunk_base <= chunk) lo = mid;
    else hi = mid - 1;
  }
  const ValJob& J = jobs[lo];
  const int64_t e0 = (chunk - J.chunk_base) * kValChunk;
  const int64_t e1 = min<int64_t>(J.nelem, e0 + kValChunk);
  double s = 0.0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const double d = double(J.c32[e]) - J.c64[e];
    const double dd = d * d;
    s += dd;
  }
  s = block_sum_f64(s, red);
  if (threadIdx.x == 0) partial[chunk] = s;
}

__global__ void k_val_final(const ValJob* __restrict__ jobs, int njobs, int64_t nchunks,
                            const double* __restrict__ partial, double* __restrict__ out) {
  const int j = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= njobs) return;
  const int64_t end = j + 1 < njobs ? jobs[j + 1].chunk_base : nchunks;
  double s = 0.0;
  for (int64_t q = jobs[j].chunk_base; q < end; ++q) s += partial[q];
  out[j] = s;
}

hipError_t launch_validate(hipStream_t s, const ValJob* jobs, int njobs, int64_t nchunks, double* partial,
                           double* out) {
  if (njobs == 0) return hipSuccess;
  if (nchunks > 0) {
    hipLaunchKernelGGL(k_val_partial, dim3(uint32_t(nchunks)), dim3(256), 0, s, jobs, njobs, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_val_final, dim3(uint32_t((njobs + 63) / 64)), dim3(64), 0, s, jobs, njobs, nchunks, partial,
                     out);
  return hipGetLastError();
}

// (I, K, J) triples of a product's plan, for parity checks.
__global__ void k_decode_kept(int G, const int64_t* __restrict__ off, const int2* __restrict__ pairs,
                              int64_t aoff, const int32_t* __restrict__ akeys, int32_t* __restrict__ ijk) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= int64_t(G) * G) return;
  uint32_t i, j;
  demorton(uint32_t(c), i, j);
  for (int64_t t = off[c]; t < off[c + 1]; ++t) {
    uint32_t ai, ak;
    demorton(uint32_t(akeys[pairs[t].x - aoff]), ai, ak);
    ijk[3 * t] = int32_t(i);
    ijk[3 * t + 1] = int32_t(ak);
    ijk[3 * t + 2] = int32_t(j);
  }
}

hipError_t launch_decode_kept(hipStream_t s, int G, const int64_t* off, const int2* pairs, int64_t aoff,
                              const int32_t* akeys, int32_t* ijk) {
  const int64_t G2 = int64_t(G) * G;
  hipLaunchKernelGGL(k_decode_kept, dim3(uint32_t((G2 + 255) / 256)), dim3(256), 0, s, G, off, pairs, aoff, akeys,
                     ijk);
  return hipGetLastError();
}

}  // namespace spamm
